// Plan setup, pipeline orchestration and the C ABI (include/helm.h).
//
// 2D (Section 4.2), with x_1 periodised and lines along x_2:
//   f^   = F_1 f / mu_1                                      (eq. (step1FFTfcoeff), forward DFT)
//   Step 1: z1_l = (T^B_l)^{-1} f^_l, v_b = boundary rows of F_1^{-1} z1     (eqs. (2dLUBs1), (2dBs1))
//   Step 2: r = C v_b, z2_l = (T^A_l)^{-1} (V_1^b)^T r, w_b = V_1^b z2       (eqs. (step2-1)-(step2-3))
//   Step 3: q = C (v_b + w_b), z3_l = (T^B_l)^{-1} (f^_l + h^_l)             (eqs. (step3term), (2dLUBs3))
//           u = F_1^{-1} z3                                                  (eq. (step3IFFTz3coeff))
// 3D (Section 5.2): the same three steps along x_1, each block solve being the
// 2D method along x_2 on the shifted problems of eqs. (A2D2)-(B2D2aux); by
// linearity the x_2 transform of every right-hand side is taken once (the
// whole array for f^, two planes for the boundary terms), and the outer
// boundary reductions act on the inner solutions in x_2-mode space before a
// two-plane inverse transform.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <cstdio>
#include <cstdlib>

#include "helm_internal.h"

namespace helm {

namespace {

bool is_pow2(int64_t n) { return n >= 2 && (n & (n - 1)) == 0; }

// h times the corner entry 1/h + g of a 1D stiffness matrix (face condition
// du/dn + g u = 0).
double2 corner_h(double2 g, double h) { return make_double2(1.0 + h * g.x, h * g.y); }

struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    // the old buffer may still be in use by queued work (a graph launched
    // earlier, an asynchronous solve): let it drain before freeing
    if (p) (void)hipDeviceSynchronize();
    release();
    if (b == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = b;
    return hipSuccess;
  }
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

struct Roots {  // e^{sign 2 pi i t / L}, t < L, in double and float
  DevMem d, f;
};

// Periodised axis: closed-form periodic spectra (eqs. (eigvectorsPer),
// (eigvaluesPer)) and the absorbing-boundary eigenpairs (eq. (EVP1a)).
struct PAxis {
  int n = 0;
  double h = 0;
  double2 glo{0, 0}, ghi{0, 0};  // face coefficients g of du/dn + g u = 0
  std::vector<cd> lamA, va0, va1;
  // spectra to extended precision (host), for the shifted values below
  std::vector<long double> lamBx;
  std::vector<std::complex<long double>> lamAx;
  DevMem tab;  // all per-mode tables below, one allocation
  // sigB / sigA: lambda - w^2 of the periodic / absorbing spectra, formed in
  // extended precision and rounded once
  double2 *sigB = nullptr, *sigA = nullptr, *genB0 = nullptr, *genB1 = nullptr, *redB0 = nullptr,
          *redB1 = nullptr, *va0d = nullptr, *va1d = nullptr;
  double* invmu = nullptr;
  BDiff bd;
  int na = 0, nbp = 0;  // FFT split n = na * nbp (nbp = first pass length); na = 1 -> one pass
  // Bluestein (chirp-z) transform for lengths that are not powers of two:
  // convolution length M >= 2n - 1 (a power of two, or 9 * 2^j) split as
  // Mna * Mnbp (Mna = 9 in the second case).
  int blue = 0, M = 0, Mna = 0, Mnbp = 0;
  int onepass = 0;  // the whole chirp-z convolution in one pass (tuned)
  DevMem btab;
  const void* chirp_d[2] = {nullptr, nullptr};  // w for sign -1, +1 (double2[n])
  const void* chirp_f[2] = {nullptr, nullptr};  // same in float2
  const void* bhat_d[2] = {nullptr, nullptr};   // FFT_M of the convolution kernel (double2[M])
  const void* bhat_f[2] = {nullptr, nullptr};
  // full absorbing-boundary eigenvectors for the dense transform:
  // V[i][l] = v_l(i) and its transpose, interleaved complex, double and float
  DevMem vmat;
  const void *Vd = nullptr, *VTd = nullptr, *Vf = nullptr, *VTf = nullptr;
};

}  // namespace

}  // namespace helm

struct helm_plan {
  int dim = 0;
  int64_t grid[3] = {0, 0, 0};
  double h[3] = {0, 0, 0};
  // operator -Lap u - c u with face conditions du/dn + g u = 0: c (and c to
  // extended precision, for the shifts), g per axis and face
  double cz = 0;
  long double czx = 0;
  double2 glo[3] = {}, ghi[3] = {};
  helm_options opt{};
  int device = 0;
  helm::PAxis ax[2];
  int nper = 0;  // periodised axes: 1 (2D) or 2 (3D)
  // last (line) axis
  int nL = 0;
  double hL = 0;
  double2 kLo{1, 0}, kHi{1, 0};
  std::map<int, helm::Roots> roots_fwd, roots_inv;
  // workspace
  int cap_rhs = 0;
  int cap_prec = -1;
  helm::DevMem W0, W1, W2, R, part, VB, PIb, P0, P1, P2, P3, scratch, norms, BT1;
  // LU factor tables (reciprocal Thomas pivots) per line-matrix family
  // (outer branch, inner branch): [0] = (B, B), [1] = (B, A), [2] = (A, B),
  // [3] = (A, A); 2D uses [0], [1].
  helm::DevMem factors;
  const double2* seed[4] = {nullptr, nullptr, nullptr, nullptr};
  // per family, sigma of every line matrix [nO][nI] (same family order)
  helm::DevMem sigtab;
  const double2* sig[4] = {nullptr, nullptr, nullptr, nullptr};
  // device-side refinement control (IrCtl) for captured solves
  helm::DevMem ctl;
  int dense = 0;  // 1: periodised axes use the dense eigenvector transforms
  // Boundary operator tables (3D, helm_options.boundary): capW holds the
  // inner Step-2 map of every outer periodic mode l (line family (B, A)),
  // capH the outer Step-2 map of every inner absorbing mode m (family
  // (A, A)); each as two blocks T_{k'}[g][x'][k][x] (cap.hip).  Solves of at
  // least cap_min_nb right-hand sides use them (0: never).
  helm::DevMem capW, capH;
  const void *capW0 = nullptr, *capW1 = nullptr, *capH0 = nullptr, *capH1 = nullptr;
  int cap_fp32 = 0;  // tables in complex64 (mixed-precision plans)
  int cap_min_nb = 0;
  int red_layout = 2;  // layout of the line reductions over the outer modes (2 or 3)
  int fft_small = 0;   // 512-point passes: 0 the 128 KB tile, 1 the 64 KB complex64 tile, 2 streaming (tuned)
  double cap_ms[4] = {-1, -1, -1, -1};  // measured: lines at 1 and 16 RHS, tables at 1 and 16 RHS
  std::string tune_path;
  double tune_ms[2] = {-1.0, -1.0};  // measured FFT / dense solve times (AUTO)
  std::vector<double> h_norms;
  // pinned host copy of the residual norms for solves that may not allocate
  // ([2 * HELM_STATIC_MAX_RHS], allocated at setup)
  double* h_norms_pin = nullptr;
  // set while helm_solve_static runs: nothing may be allocated
  bool no_alloc = false;
  // this device's address of the static workspace array (helm_solve_static)
  void* static_ws = nullptr;
  helm_report rep{};
  // per-kernel event timing
  struct Ev {
    hipEvent_t a, b;
    int cls;
    double bytes;
  };
  bool prof = false;
  // device flag read by every launch while set (captured refinement steps)
  const int* skip_cur = nullptr;
  std::vector<Ev> evs;
  size_t nev = 0;
  helm_kernel_stats kst{};
  // Workspace generation: raised whenever a workspace buffer moves, so that
  // graphs captured on the old addresses are not launched again.
  uint64_t ws_gen = 0;
  // Captured solve for repeated helm_solve calls on unchanged arguments:
  // the arguments of the previous call and the refinement steps it took,
  // the graph with the arguments it was captured for, and a pinned host
  // copy of the device refinement control written by its last launch.
  struct Key {
    const void* f = nullptr;
    void* u = nullptr;
    int nrhs = 0;
    hipStream_t st = nullptr;
    bool operator==(const Key& o) const { return f == o.f && u == o.u && nrhs == o.nrhs && st == o.st; }
  };
  Key last_key, graph_key;
  int prev_steps = -1;
  int graph_steps = 0;
  uint64_t graph_gen = 0;
  hipStream_t gcap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  void* ctl_host = nullptr;
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  ~helm_plan() {
    drop_graph();
    if (gcap) (void)hipStreamDestroy(gcap);
    if (ctl_host) (void)hipHostFree(ctl_host);
    if (h_norms_pin) (void)hipHostFree(h_norms_pin);
    for (auto& e : evs) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
  }
};

namespace helm {

namespace {

hipError_t upload(void* dst, const void* src, size_t bytes) {
  return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
}

int map_err(hipError_t e) {
  if (e == hipSuccess) return HELM_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return HELM_ENOMEM;
  return HELM_EDEVICE;
}

#define HCHK(expr)                      \
  do {                                  \
    hipError_t _e = (expr);             \
    if (_e != hipSuccess) return map_err(_e); \
  } while (0)

// Kernel slots of helm_kernel_stats.
enum KSlot {
  K_FFT64 = 0, K_FFT32 = 1, K_LINES = 2, K_INNER_MID = 3, K_SUM = 4, K_OUTER_MID = 5, K_RESID = 6, K_DENSE = 7,
  K_CAP = 8
};

// Launch through `fn` (returning hipError_t), bracketed by events if profiling.
template <class F> hipError_t timed(helm_plan* p, int cls, double bytes, hipStream_t st, F&& fn) {
  if (!p->prof) return fn();
  if (p->nev == p->evs.size()) {
    helm_plan::Ev e;
    hipError_t r = hipEventCreate(&e.a);
    if (r != hipSuccess) return r;
    r = hipEventCreate(&e.b);
    if (r != hipSuccess) return r;
    p->evs.push_back(e);
  }
  helm_plan::Ev& e = p->evs[p->nev++];
  e.cls = cls;
  e.bytes = bytes;
  hipError_t r = hipEventRecord(e.a, st);
  if (r != hipSuccess) return r;
  r = fn();
  if (r != hipSuccess) return r;
  return hipEventRecord(e.b, st);
}

hipError_t collect_events(helm_plan* p) {
  for (size_t i = 0; i < p->nev; ++i) {
    helm_plan::Ev& e = p->evs[i];
    hipError_t r = hipEventSynchronize(e.b);
    if (r != hipSuccess) return r;
    float ms = 0.f;
    r = hipEventElapsedTime(&ms, e.a, e.b);
    if (r != hipSuccess) return r;
    p->kst.ms[e.cls] += ms;
    p->kst.bytes[e.cls] += e.bytes;
    p->kst.calls[e.cls] += 1;
  }
  p->nev = 0;
  return hipSuccess;
}

size_t esz_of(int kind) { return kind == ST_C64 ? sizeof(float2) : sizeof(double2); }

// In-place radix-2 DFT of a power-of-two length on the host (FP64), sign -1
// forward; used once per plan for the transformed Bluestein kernel.
void host_fft(std::vector<cd>& x, int sign) {
  const int n = (int)x.size();
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(x[i], x[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    for (int k = 0; k < len / 2; ++k) {
      const double th = sign * 2.0 * M_PI * k / len;
      const cd w(std::cos(th), std::sin(th));
      for (int i = 0; i < n; i += len) {
        const cd u = x[i + k], v = x[i + k + len / 2] * w;
        x[i + k] = u + v;
        x[i + k + len / 2] = u - v;
      }
    }
  }
}

// DFT of any length of the form 2^j m with small odd m (here m = 1 or 9):
// radix-2 decimation in time down to the odd length, which is summed
// directly.  Host-side, for plan tables only.
void host_dft(std::vector<cd>& x, int sign) {
  const int n = (int)x.size();
  if ((n & (n - 1)) == 0) {
    host_fft(x, sign);
    return;
  }
  if (n % 2) {
    std::vector<cd> y(n);
    for (int k = 0; k < n; ++k) {
      cd acc(0.0);
      for (int j = 0; j < n; ++j) {
        const double th = sign * 2.0 * M_PI * (double)(((int64_t)j * k) % n) / n;
        acc += x[j] * cd(std::cos(th), std::sin(th));
      }
      y[k] = acc;
    }
    x = y;
    return;
  }
  std::vector<cd> e(n / 2), o(n / 2);
  for (int j = 0; j < n / 2; ++j) {
    e[j] = x[2 * j];
    o[j] = x[2 * j + 1];
  }
  host_dft(e, sign);
  host_dft(o, sign);
  for (int k = 0; k < n / 2; ++k) {
    const double th = sign * 2.0 * M_PI * k / n;
    const cd t = o[k] * cd(std::cos(th), std::sin(th));
    x[k] = e[k] + t;
    x[k + n / 2] = e[k] - t;
  }
}

void pow2_split(int L, int* na, int* nb) {
  if (L <= 512) {
    *na = 1;
    *nb = L;
    return;
  }
  int b = 1;
  while ((int64_t)b * b < L) b <<= 1;
  *nb = b;
  *na = L / b;
}

// Bluestein tables of a periodised axis of length n (not a power of two):
// chirp w_s[j] = e^{s pi i (j^2 mod 2n)/n} and the length-M forward DFT of the
// kernel b_s[m] = e^{-s pi i m^2/n} (m in (-n, n), wrapped modulo M), s = -1, +1.
// The convolution length M >= 2n - 1 is the smaller of the next power of two
// and 9 * 2^j >= 576, split as nb (the passes that carry the chirps, a power
// of two, 64 <= nb <= 512) times na = 9 * 2^k <= 72 (the convolution pass):
// for the paper's n = 2^k + 1 that is 2.25 n instead of 4 n.
int setup_bluestein(PAxis& a) {
  const int n = a.n;
  int M = 1;
  while (M < 2 * n - 1) M <<= 1;
  if (M > 512 * 512) return HELM_EUNSUPPORTED;
  int M9 = 9;
  while (M9 < 2 * n - 1) M9 <<= 1;
  a.blue = 1;
  if (M9 < M && M9 >= 576 && M9 <= 72 * 512) {
    M = M9;
    a.Mnbp = M9 <= 4608 ? 64 : M9 / 72;
    a.Mna = M9 / a.Mnbp;
  } else {
    pow2_split(M, &a.Mna, &a.Mnbp);
  }
  a.M = M;
  std::vector<double2> hd((size_t)2 * n + 2 * M);
  std::vector<float2> hf((size_t)2 * n + 2 * M);
  for (int si = 0; si < 2; ++si) {
    const int sg = si == 0 ? -1 : 1;
    std::vector<cd> b(M, cd(0.0));
    for (int64_t j = 0; j < n; ++j) {
      const int64_t jj = (j * j) % (2 * (int64_t)n);
      const double th = M_PI * (double)jj / n;
      const cd w(std::cos(th), sg * std::sin(th));
      hd[(size_t)si * n + j] = hd2(w);
      b[j] = std::conj(w);
      if (j > 0) b[M - j] = std::conj(w);
    }
    host_dft(b, -1);
    for (int k = 0; k < M; ++k) hd[(size_t)2 * n + (size_t)si * M + k] = hd2(b[k]);
  }
  for (size_t i = 0; i < hd.size(); ++i) hf[i] = make_float2((float)hd[i].x, (float)hd[i].y);
  const size_t bd = hd.size() * sizeof(double2), bf = hf.size() * sizeof(float2);
  if (a.btab.ensure(bd + bf) != hipSuccess) return HELM_ENOMEM;
  if (upload(a.btab.p, hd.data(), bd) != hipSuccess) return HELM_EDEVICE;
  if (upload((char*)a.btab.p + bd, hf.data(), bf) != hipSuccess) return HELM_EDEVICE;
  const double2* d = a.btab.as<double2>();
  const float2* f = reinterpret_cast<const float2*>((char*)a.btab.p + bd);
  for (int si = 0; si < 2; ++si) {
    a.chirp_d[si] = d + (size_t)si * n;
    a.bhat_d[si] = d + 2 * (size_t)n + (size_t)si * M;
    a.chirp_f[si] = f + (size_t)si * n;
    a.bhat_f[si] = f + 2 * (size_t)n + (size_t)si * M;
  }
  return HELM_OK;
}

Roots* get_roots(helm_plan* p, int L, int sign) {
  auto& mp = sign < 0 ? p->roots_fwd : p->roots_inv;
  auto it = mp.find(L);
  if (it != mp.end()) return &it->second;
  if (p->no_alloc) return nullptr;  // every table is built at setup (prepare_roots)
  Roots& r = mp[L];
  std::vector<double2> hd(L);
  std::vector<float2> hf(L);
  for (int t = 0; t < L; ++t) {
    // angle 2 pi t / L reduced to the first octant symmetry-free form
    const double th = 2.0 * M_PI * (double)t / (double)L;
    const double c = std::cos(th), s = sign * std::sin(th);
    hd[t] = make_double2(c, s);
    hf[t] = make_float2((float)c, (float)s);
  }
  if (r.d.ensure(L * sizeof(double2)) != hipSuccess || r.f.ensure(L * sizeof(float2)) != hipSuccess) return nullptr;
  if (upload(r.d.p, hd.data(), L * sizeof(double2)) != hipSuccess) return nullptr;
  if (upload(r.f.p, hf.data(), L * sizeof(float2)) != hipSuccess) return nullptr;
  return &r;
}

void radix_plan(int L, FftPass& f) {
  const bool m9 = L % 9 == 0;
  const int L2 = m9 ? L / 9 : L;
  int p = 0;
  while ((1 << p) < L2) ++p;
  f.nst = 0;
  const int rem = p % 3;
  if (rem == 1) f.radix[f.nst++] = 2;
  if (rem == 2) f.radix[f.nst++] = 4;
  for (int i = 0; i < p / 3; ++i) f.radix[f.nst++] = 8;
  if (m9) f.radix[f.nst++] = 3, f.radix[f.nst++] = 3;
}

// Build every table of roots of unity the transforms of this plan use, so
// that solves find them in place (and solves that may not allocate can run).
int prepare_roots(helm_plan* p) {
  for (int j = 0; j < p->nper; ++j) {
    const PAxis& a = p->ax[j];
    std::vector<int> lens;
    if (!a.blue) {
      lens = {a.n};
      if (a.na > 1) lens.insert(lens.end(), {a.na, a.nbp});
    } else {
      lens = {a.M};
      if (a.Mna > 1) lens.insert(lens.end(), {a.Mna, a.Mnbp});
    }
    for (int L : lens)
      for (int sign : {-1, +1})
        if (!get_roots(p, L, sign)) return HELM_ENOMEM;
  }
  return HELM_OK;
}

int pick_W(int L, int64_t, bool fp32) { return fft_tile_width(L, fp32); }

// A transform pass with the plan's tile choice.
FftPass with_tile(const helm_plan* p, FftPass f) {
  f.small_tile = p->fft_small;
  return f;
}

// Power-of-two DFT of length L along the axis of [O][L][S] data (S
// contiguous): one pass for L <= 512, else the four-step split L = na * nb
// (pass 1 writes `tmp`).  Per-mode complex multiplier `cmode`, real `scale`.
int run_pow2(helm_plan* p, int L, int na, int nb, int sign, bool fp32, const void* in, int in_kind, void* out,
             int out_kind, int64_t O, int64_t S, const double* scale, double scale_c, const void* cmode,
             int accumulate, void* tmp, int tmp_kind, const int* skip, hipStream_t st) {
  if (na <= 1) {
    Roots* r = get_roots(p, L, sign);
    if (!r) return HELM_ENOMEM;
    FftPass f;
    f.L = L;
    radix_plan(L, f);
    f.I = S;
    f.O = O;
    f.od = 1;
    f.in_so = (int64_t)L * S;
    f.in_sj = S;
    f.out_so1 = (int64_t)L * S;
    f.out_so2 = 0;
    f.out_sk = S;
    f.W = pick_W(L, S, fp32);
    f.in_kind = in_kind;
    f.out_kind = out_kind;
    f.accumulate = accumulate;
    f.sign = sign;
    f.scale = scale;
    f.scale_c = scale_c;
    f.cmode = cmode;
    f.skip = skip ? skip : p->skip_cur;
    f.tw = fp32 ? r->f.p : r->d.p;
    const double by = (double)O * L * S * (esz_of(in_kind) + esz_of(out_kind));
    HCHK(timed(p, fp32 ? K_FFT32 : K_FFT64, by, st, [&] { return launch_fft_pass(with_tile(p, f), fp32, in, out, st); }));
    return HELM_OK;
  }
  // four-step: L = na * nb, x = a + na b, k = c + nb d
  Roots* r1 = get_roots(p, nb, sign);
  Roots* r2 = get_roots(p, na, sign);
  Roots* rn = get_roots(p, L, sign);
  if (!r1 || !r2 || !rn) return HELM_ENOMEM;
  FftPass f1;
  f1.L = nb;
  radix_plan(nb, f1);
  f1.I = (int64_t)na * S;
  f1.O = O;
  f1.od = 1;
  f1.in_so = (int64_t)L * S;
  f1.in_sj = (int64_t)na * S;
  f1.out_so1 = (int64_t)L * S;
  f1.out_sk = (int64_t)na * S;
  f1.tw4_S = S;
  f1.tw4_n = L;
  f1.W = pick_W(nb, f1.I, fp32);
  f1.in_kind = in_kind;
  f1.out_kind = tmp_kind;
  f1.sign = sign;
  f1.skip = skip ? skip : p->skip_cur;
  f1.tw = fp32 ? r1->f.p : r1->d.p;
  f1.tw4 = fp32 ? rn->f.p : rn->d.p;
  const double by1 = (double)O * L * S * (esz_of(in_kind) + esz_of(tmp_kind));
  HCHK(timed(p, fp32 ? K_FFT32 : K_FFT64, by1, st, [&] { return launch_fft_pass(with_tile(p, f1), fp32, in, tmp, st); }));
  FftPass f2;
  f2.L = na;
  radix_plan(na, f2);
  f2.I = S;
  f2.O = O * nb;
  f2.od = nb;
  f2.in_so = (int64_t)na * S;
  f2.in_sj = S;
  f2.out_so1 = (int64_t)L * S;
  f2.out_so2 = S;
  f2.out_sk = (int64_t)nb * S;
  f2.W = pick_W(na, S, fp32);
  f2.in_kind = tmp_kind;
  f2.out_kind = out_kind;
  f2.accumulate = accumulate;
  f2.sign = sign;
  f2.scale = scale;
  f2.scale_c = scale_c;
  f2.cmode = cmode;
  f2.skip = skip ? skip : p->skip_cur;
  f2.tw = fp32 ? r2->f.p : r2->d.p;
  const double by2 = (double)O * L * S * (esz_of(tmp_kind) + esz_of(out_kind));
  HCHK(timed(p, fp32 ? K_FFT32 : K_FFT64, by2, st, [&] { return launch_fft_pass(with_tile(p, f2), fp32, tmp, out, st); }));
  return HELM_OK;
}

// DFT along a periodised axis of data [O][n][S] (S contiguous).
// Forward: sign -1 and per-mode scale 1/mu (if scale), inverse: sign +1, 1/n.
// Lengths that are not powers of two use Bluestein's chirp-z algorithm:
// jk = (j^2 + k^2 - (k - j)^2)/2 turns the DFT into a convolution with the
// chirp kernel, evaluated with transforms of length M >= 2n - 1 (a power of
// two, or 9 * 2^j as a length-2^j pass and a length-9 convolution pass).
// The chirp multiplications are folded into the first load and the last
// store, and the convolution's middle (forward pass, kernel product, inverse
// pass) is one kernel, so a transform costs n + M + 2M + M + n element moves
// (M <= 512: n + M + M + n) in the plan's temporary BT1.
int run_fft(helm_plan* p, const PAxis& a, int sign, bool fp32, const void* in, int in_kind, void* out,
            int out_kind, int64_t O, int64_t S, const double* scale, double scale_c, int accumulate,
            void* tmp, int tmp_kind, hipStream_t st, const int* skip = nullptr) {
  if (!a.blue)
    return run_pow2(p, a.n, a.na, a.nbp, sign, fp32, in, in_kind, out, out_kind, O, S, scale, scale_c,
                    nullptr, accumulate, tmp, tmp_kind, skip, st);
  (void)tmp;
  (void)tmp_kind;
  const int si = sign < 0 ? 0 : 1;
  const int T = fp32 ? ST_C64 : ST_C128;
  const int64_t n = a.n, M = a.M;
  void* t1 = p->BT1.p;
  const void* chirp = fp32 ? a.chirp_f[si] : a.chirp_d[si];
  const void* bhat = fp32 ? a.bhat_f[si] : a.bhat_d[si];
  const int* sk = skip ? skip : p->skip_cur;
  const int K = fp32 ? K_FFT32 : K_FFT64;
  if (a.onepass) {
    // one pass: the M-point DFT of the chirped rows (zero past n) in LDS,
    // the product with the transformed kernel, the unscaled inverse DFT
    // (conj(DFT(conj(.)))), rows < n stored with the chirp, the per-mode
    // scale and 1/M
    Roots* rf = get_roots(p, (int)M, -1);
    if (!rf) return HELM_ENOMEM;
    FftPass f;
    f.L = (int)M;
    radix_plan((int)M, f);
    f.I = S;
    f.O = O;
    f.od = 1;
    f.in_so = n * S;
    f.in_sj = S;
    f.out_so1 = n * S;
    f.out_sk = S;
    f.in_kind = in_kind;
    f.out_kind = out_kind;
    f.sign = -1;
    f.tw = fp32 ? rf->f.p : rf->d.p;
    f.cin = chirp;
    f.cout = chirp;
    f.chirp_n = n;
    f.chirp_na = 1;
    f.chirp_S = S;
    f.cmode = bhat;
    f.conj_out = 1;
    f.scale = scale;
    f.scale_c = scale_c / (double)M;
    f.accumulate = accumulate;
    f.skip = sk;
    const double by = (double)O * S * n * (esz_of(in_kind) + esz_of(out_kind) * (accumulate ? 2 : 1));
    HCHK(timed(p, K, by, st, [&] { return launch_conv_pass(f, fp32, in, out, st); }));
    return HELM_OK;
  }
  if (a.Mna <= 1) {
    Roots* rf = get_roots(p, (int)M, -1);
    Roots* ri = get_roots(p, (int)M, +1);
    if (!rf || !ri) return HELM_ENOMEM;
    FftPass f;
    f.L = (int)M;
    radix_plan((int)M, f);
    f.I = S;
    f.O = O;
    f.od = 1;
    f.in_so = n * S;
    f.in_sj = S;
    f.out_so1 = M * S;
    f.out_sk = S;
    f.in_kind = in_kind;
    f.out_kind = T;
    f.sign = -1;
    f.tw = fp32 ? rf->f.p : rf->d.p;
    f.cin = chirp;
    f.chirp_n = n;
    f.chirp_na = 1;
    f.chirp_S = S;
    f.cmode = bhat;
    f.skip = sk;
    const double by1 = (double)O * S * ((double)n * esz_of(in_kind) + (double)M * esz_of(T));
    HCHK(timed(p, K, by1, st, [&] { return launch_fft_pass(with_tile(p, f), fp32, in, t1, st); }));
    FftPass g = f;
    g.in_so = M * S;
    g.out_so1 = n * S;
    g.in_kind = T;
    g.out_kind = out_kind;
    g.sign = +1;
    g.tw = fp32 ? ri->f.p : ri->d.p;
    g.cin = nullptr;
    g.cmode = nullptr;
    g.cout = chirp;
    g.scale = scale;
    g.scale_c = scale_c / (double)M;
    g.accumulate = accumulate;
    const double by2 = (double)O * S * ((double)M * esz_of(T) + (double)n * esz_of(out_kind) * (accumulate ? 2 : 1));
    HCHK(timed(p, K, by2, st, [&] { return launch_fft_pass(with_tile(p, g), fp32, t1, out, st); }));
    return HELM_OK;
  }
  // four-step convolution, M = na * nb: x = a + na b, k = c + nb d
  const int na = a.Mna, nb = a.Mnbp;
  Roots* rbf = get_roots(p, nb, -1);
  Roots* rbi = get_roots(p, nb, +1);
  Roots* raf = get_roots(p, na, -1);
  Roots* rMf = get_roots(p, (int)M, -1);
  Roots* rMi = get_roots(p, (int)M, +1);
  if (!rbf || !rbi || !raf || !rMf || !rMi) return HELM_ENOMEM;
  // 1: length-nb DFTs over b of the chirped input rows (zero past n), twiddle
  //    e^{-2 pi i a c / M}, into t1[o][c][a][s]
  FftPass f1;
  f1.L = nb;
  radix_plan(nb, f1);
  f1.I = (int64_t)na * S;
  f1.O = O;
  f1.od = 1;
  f1.in_so = n * S;
  f1.in_sj = (int64_t)na * S;
  f1.out_so1 = M * S;
  f1.out_sk = (int64_t)na * S;
  f1.tw4_S = S;
  f1.tw4_n = (int)M;
  f1.in_kind = in_kind;
  f1.out_kind = T;
  f1.sign = -1;
  f1.tw = fp32 ? rbf->f.p : rbf->d.p;
  f1.tw4 = fp32 ? rMf->f.p : rMf->d.p;
  f1.cin = chirp;
  f1.chirp_n = n;
  f1.chirp_na = na;
  f1.chirp_S = S;
  f1.skip = sk;
  const double by1 = (double)O * S * ((double)n * esz_of(in_kind) + (double)M * esz_of(T));
  HCHK(timed(p, K, by1, st, [&] { return launch_fft_pass(with_tile(p, f1), fp32, in, t1, st); }));
  // 2: per group c, length-na DFT over a, product with the transformed
  //    kernel at k = c + nb d, unscaled inverse over d, twiddle
  //    e^{+2 pi i c a / M}; in place
  FftPass f2;
  f2.L = na;
  radix_plan(na, f2);
  f2.I = S;
  f2.O = O * nb;
  f2.od = nb;
  f2.in_so = (int64_t)na * S;
  f2.in_sj = S;
  f2.out_so1 = M * S;
  f2.out_so2 = (int64_t)na * S;
  f2.out_sk = S;
  f2.in_kind = T;
  f2.out_kind = T;
  f2.sign = -1;
  f2.tw = fp32 ? raf->f.p : raf->d.p;
  f2.cmode = bhat;
  f2.tw4 = fp32 ? rMi->f.p : rMi->d.p;
  f2.tw4_n = (int)M;
  f2.tw4_mode = 1;
  f2.conj_out = 1;
  f2.skip = sk;
  const double by2 = (double)O * S * (double)M * 2.0 * esz_of(T);
  HCHK(timed(p, K, by2, st, [&] { return launch_conv_pass(f2, fp32, t1, t1, st); }));
  // 3: per a, length-nb inverse DFT over c, rows x = a + na b < n stored with
  //    the chirp, the per-mode scale and 1/M
  FftPass f3;
  f3.L = nb;
  radix_plan(nb, f3);
  f3.I = (int64_t)na * S;
  f3.O = O;
  f3.od = 1;
  f3.in_so = M * S;
  f3.in_sj = (int64_t)na * S;
  f3.out_so1 = n * S;
  f3.out_sk = (int64_t)na * S;
  f3.in_kind = T;
  f3.out_kind = out_kind;
  f3.sign = +1;
  f3.tw = fp32 ? rbi->f.p : rbi->d.p;
  f3.cout = chirp;
  f3.chirp_n = n;
  f3.chirp_na = na;
  f3.chirp_S = S;
  f3.scale = scale;
  f3.scale_c = scale_c / (double)M;
  f3.accumulate = accumulate;
  f3.skip = sk;
  const double by3 = (double)O * S * ((double)M * esz_of(T) + (double)n * esz_of(out_kind) * (accumulate ? 2 : 1));
  HCHK(timed(p, K, by3, st, [&] { return launch_fft_pass(with_tile(p, f3), fp32, t1, out, st); }));
  return HELM_OK;
}

// Layout of a reduction over l (red 2 or 3, see the line kernel): red 2
// gives a block one m and its slots consecutive l, red 3 gives the slots
// consecutive m at one l.  Both compute the same sums; which is faster
// depends on the shape (measured at 512^3 x 16: red 3 0.5% slower, at 256^3
// 1.5% slower, at 513^3 1% faster), so the plan times both at setup (3D) and
// keeps the faster (tune_layout); HELM_RED_L_LAYOUT=2 or 3 in the
// environment at setup fixes it instead (tests).
int red_l_mode(const helm_plan* p) { return p->red_layout; }

// Lines per tile and tiles of a line launch; `layout` (2 or 3) only matters
// for red 2.  At least 8 lines feed each partial sum (partials stay below 1/4
// of an N-sized array).  A reducing launch writes one partial of 2 nL values
// per block, so it uses about as many blocks as stay resident at once (one
// 512-thread or two 256-thread blocks per compute unit at the register use of
// the reducing kernels) and no more; other launches take up to 2048 blocks.
// Layout 3 writes one partial per slot and splits the l of every group of
// consecutive m into as few tiles as give at least 1024 blocks.
void tiles_for_layout(int red, int layout, int nb, int nO, int nI, int nL, int* tile, int* ntiles) {
  int P, c, NT;
  lines_geometry(nL, &P, &c, &NT);
  const int LPB = NT / P;
  if (red == 2 && layout == 3) {
    const int64_t groups = (int64_t)nb * ((nI + LPB - 1) / LPB);
    int64_t nt = groups >= 1024 ? 1 : (1024 + groups - 1) / groups;
    if (nt > nO) nt = nO;
    const int64_t t = (nO + nt - 1) / nt;
    *tile = (int)t;
    *ntiles = (int)((nO + t - 1) / t);
    return;
  }
  const int64_t extent = red == 1 ? nI : (red == 2 ? nO : (int64_t)nb * nO * nI);
  const int64_t groups = red == 1 ? (int64_t)nb * nO : (red == 2 ? (int64_t)nb * nI : 1);
  int64_t t = red ? 8 : LPB;
  const int64_t lines = extent * groups;
  const int64_t target = red ? (NT >= 512 ? 256 : 512) : 2048;
  if (lines / t > target) t = (lines + target - 1) / target;
  if (red && t > extent) t = extent;
  t = (t + LPB - 1) / LPB * LPB;
  *tile = (int)t;
  *ntiles = (int)((extent + t - 1) / t);
}

void tiles_for(const helm_plan* p, int red, int nb, int nO, int nI, int nL, int* tile, int* ntiles) {
  tiles_for_layout(red, red == 2 ? red_l_mode(p) : red, nb, nO, nI, nL, tile, ntiles);
}

// Partial sums of a reducing launch; for red 2 the larger of the two layouts,
// so that the buffer fits whichever layout a later solve takes.
size_t part_elems(int red, int nb, int nO, int nI, int nL) {
  int tile, nt, nt3 = 0;
  tiles_for_layout(red, 2, nb, nO, nI, nL, &tile, &nt);
  if (red == 2) tiles_for_layout(red, 3, nb, nO, nI, nL, &tile, &nt3);
  const int64_t groups = red == 1 ? (int64_t)nb * nO : (int64_t)nb * nI;
  return (size_t)groups * std::max(nt, nt3) * 2 * nL;
}

struct Level {  // geometry of one inner 2D solve, batched over (b, l)
  int nb, nO, nI, nL;
  const PAxis* inner;
  double w2;
};

// One inner three-step solve (the 2D method of Section 4.2 applied to every
// outer mode l with sigma shifted by sO[l]): S1 with reduction over m, the
// boundary operator, S2, the boundary operator, S3 (store or reduce over l).
struct InnerIO {
  const double2* sO = nullptr;
  const void* in = nullptr;
  int in_kind = ST_C128;
  const void* PO = nullptr;  // rank-2 rows, in the storage type of the lines
  int PO_kind = ST_C128;
  const double2* alpha0 = nullptr;
  const double2* alpha1 = nullptr;
  void* out = nullptr;
  int out_kind = ST_C128;
  const double2* rhoL0 = nullptr;
  const double2* rhoL1 = nullptr;
  const double2* seedB = nullptr;  // line matrices with the periodic inner branch (S1, S3)
  const double2* seedA = nullptr;  // line matrices with the absorbing inner branch (S2)
  const double2* sigTB = nullptr;  // their sigma tables
  const double2* sigTA = nullptr;
  bool capS2 = false;  // Step 2 from the plan's table capW instead of a line sweep
};

// Product of a boundary operator table with nb pairs of boundary vectors
// (cap.hip), timed with the table bytes it streams.
int cap_apply(helm_plan* p, const void* T0, const void* T1, int nb, int G, const double2* in,
              int64_t in_b, int64_t in_g, int64_t in_k, double2* out, int64_t out_b, int64_t out_g, int64_t out_k,
              hipStream_t st) {
  CapArgs ca;
  ca.nb = nb;
  ca.G = G;
  ca.nL = p->nL;
  ca.T0 = T0;
  ca.T1 = T1;
  ca.t_fp32 = p->cap_fp32;
  ca.in = in;
  ca.in_b = in_b;
  ca.in_g = in_g;
  ca.in_k = in_k;
  ca.out = out;
  ca.out_b = out_b;
  ca.out_g = out_g;
  ca.out_k = out_k;
  ca.skip = p->skip_cur;
  const double by = 2.0 * G * (2.0 * p->nL) * p->nL * (p->cap_fp32 ? sizeof(float2) : sizeof(double2)) *
                    ((nb + 15) / 16);
  HCHK(timed(p, K_CAP, by, st, [&] { return launch_cap_apply(ca, st); }));
  return HELM_OK;
}

int inner_solve(helm_plan* p, const Level& lv, const InnerIO& io, hipStream_t st) {
  const PAxis& I = *lv.inner;
  const double2 sC = make_double2(-lv.w2, 0.0);
  LineArgs base;
  base.skip = p->skip_cur;
  base.nb = lv.nb;
  base.nO = lv.nO;
  base.nI = lv.nI;
  base.nL = lv.nL;
  base.sO = io.sO;
  base.sC = sC;
  base.hL = p->hL;
  base.kLo = p->kLo;
  base.kHi = p->kHi;
  base.piv = io.seedB;
  base.sTab = io.sigTB;
  double2* part = p->part.as<double2>();
  const double elems = (double)lv.nb * lv.nO * lv.nI * lv.nL;
  int tile, nt;
  tiles_for(p, 1, lv.nb, lv.nO, lv.nI, lv.nL, &tile, &nt);

  // S1: (T^B)^{-1} of the right-hand side, reduced to the two boundary rows.
  LineArgs s1 = base;
  s1.sI = I.sigB;
  s1.in = io.in;
  s1.in_kind = io.in_kind;
  s1.PO = io.PO;
  s1.r2_kind = io.PO_kind;
  s1.alpha0 = io.alpha0;
  s1.alpha1 = io.alpha1;
  s1.red = 1;
  s1.rho0 = I.redB0;
  s1.rho1 = I.redB1;
  s1.part = part;
  s1.tile = tile;
  s1.ntiles = nt;
  HCHK(timed(p, K_LINES, io.in ? elems * esz_of(io.in_kind) : 0.0, st, [&] { return launch_lines(s1, st); }));

  InnerMidArgs m;
  m.skip = p->skip_cur;
  m.nb = lv.nb;
  m.nO = lv.nO;
  m.nL = lv.nL;
  m.ntiles = nt;
  m.part = part;
  m.vb_in = nullptr;
  m.vb_out = p->VB.as<double2>();
  m.out = p->PIb.as<double2>();
  m.sO = io.sO;                                  // lambda_outer - w^2 (3D) or none
  m.sC = io.sO ? make_double2(0.0, 0.0) : sC;   // p_l = -(sO[l] + sC)
  m.d = I.bd;
  m.hL = p->hL;
  m.kLo = p->kLo;
  m.kHi = p->kHi;
  HCHK(timed(p, K_INNER_MID, (double)lv.nb * lv.nO * 2 * lv.nL * sizeof(double2) * (nt + 2), st,
             [&] { return launch_inner_mid(m, st); }));

  // S2: partial solution with the absorbing-boundary eigenvectors, as a
  // line sweep or from the table of its map (one partial per (b, l))
  if (io.capS2) {
    const int64_t per = 2 * (int64_t)lv.nL, gs = (int64_t)lv.nO * per;
    const int rc2 = cap_apply(p, p->capW0, p->capW1, lv.nb, lv.nO, p->PIb.as<double2>(), gs, per, lv.nL, part, gs,
                              per, lv.nL, st);
    if (rc2) return rc2;
    m.ntiles = 1;
  } else {
    LineArgs s2 = base;
    s2.sI = I.sigA;
    s2.piv = io.seedA;
    s2.sTab = io.sigTA;
    s2.PI = p->PIb.p;  // complex128: the launch has no line storage
    s2.r2_kind = ST_C128;
    s2.beta0 = I.va0d;
    s2.beta1 = I.va1d;
    s2.red = 1;
    s2.rho0 = I.va0d;
    s2.rho1 = I.va1d;
    s2.part = part;
    s2.tile = tile;
    s2.ntiles = nt;
    HCHK(timed(p, K_LINES, 0.0, st, [&] { return launch_lines(s2, st); }));
  }

  // the Step-3 launch reads these rows (PI) in its lines' storage type
  const int k3 = io.in ? io.in_kind : (io.out ? io.out_kind : ST_C128);
  m.vb_in = p->VB.as<double2>();
  m.vb_out = nullptr;
  m.out_c64 = k3 == ST_C64;
  HCHK(timed(p, K_INNER_MID, (double)lv.nb * lv.nO * 2 * lv.nL * sizeof(double2) * (m.ntiles + 2), st,
             [&] { return launch_inner_mid(m, st); }));

  // S3: corrected periodic solve.
  LineArgs s3 = base;
  s3.sI = I.sigB;
  s3.in = io.in;
  s3.in_kind = io.in_kind;
  s3.PO = io.PO;
  s3.r2_kind = k3;  // PIb as stored above; PO was stored the same way
  if (io.PO && io.PO_kind != k3) return HELM_EINVAL;
  s3.alpha0 = io.alpha0;
  s3.alpha1 = io.alpha1;
  s3.PI = p->PIb.p;
  s3.beta0 = I.genB0;
  s3.beta1 = I.genB1;
  if (io.rhoL0) {
    int tl, ntl;
    tiles_for(p, 2, lv.nb, lv.nO, lv.nI, lv.nL, &tl, &ntl);
    s3.red = red_l_mode(p);
    s3.rho0 = io.rhoL0;
    s3.rho1 = io.rhoL1;
    s3.part = part;
    s3.tile = tl;
    s3.ntiles = ntl;
  } else {
    int tl, ntl;
    tiles_for(p, 0, lv.nb, lv.nO, lv.nI, lv.nL, &tl, &ntl);
    s3.out = io.out;
    s3.out_kind = io.out_kind;
    s3.tile = tl;
    s3.ntiles = ntl;
    if (io.PO) {
      // mode tiles of e outer x e/2 inner modes, e chosen so that a tile has
      // no more lines than the consecutive runs would have (the launch keeps
      // its number of blocks): the rank-2 rows of an inner mode are then
      // re-read once per tile instead of once per outer mode, and with the
      // XCD-major tile order the blocks resident on one XCD share the rows
      // of their inner-mode tile in L2 (512^3 x 16 storing launch: fetch 52
      // GB untiled, 48 GB with 32 x 32 tiles, 39 GB with 32 x 16)
      int P, c, NT;
      lines_geometry(lv.nL, &P, &c, &NT);
      int e = 32;
      while (e > 4 && (e * e / 2 > tl || e > lv.nO || e / 2 > lv.nI)) e /= 2;
      if (e >= 8 && (e * e / 2) % (NT / P) == 0) {
        s3.tile_l = e;
        s3.tile_m = e / 2;
      }
    }
  }
  const double by3 = (io.in ? elems * esz_of(io.in_kind) : 0.0) + (io.out ? elems * esz_of(io.out_kind) : 0.0);
  HCHK(timed(p, K_LINES, by3, st, [&] { return launch_lines(s3, st); }));
  return HELM_OK;
}

// Sum reduce-over-l partials [b][m][t][k][x] into planes [b][k][m][x].
__global__ void sum_to_planes_kernel(const double2* __restrict__ part, int nb, int nI, int nL, int ntiles,
                                     double2* __restrict__ out, const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)nb * 2 * nI * nL;
  if (i >= total) return;
  const int64_t x = i % nL;
  const int64_t m = (i / nL) % nI;
  const int64_t k = (i / ((int64_t)nL * nI)) % 2;
  const int64_t b = i / ((int64_t)nL * nI * 2);
  const double2* pp = part + ((b * nI + m) * ntiles) * 2 * nL + k * nL + x;
  double2 s = make_double2(0, 0);
  for (int t = 0; t < ntiles; ++t) s = cadd(s, pp[(int64_t)t * 2 * nL]);
  out[i] = s;
}

int sum_to_planes(helm_plan* p, const Level& lv, double2* out, hipStream_t st) {
  int tl, ntl;
  tiles_for(p, 2, lv.nb, lv.nO, lv.nI, lv.nL, &tl, &ntl);
  const int64_t total = (int64_t)lv.nb * 2 * lv.nI * lv.nL;
  HCHK(timed(p, K_SUM, (double)total * sizeof(double2) * (ntl + 1), st, [&] {
    hipLaunchKernelGGL(sum_to_planes_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       p->part.as<double2>(), lv.nb, lv.nI, lv.nL, ntl, out, p->skip_cur);
    return hipGetLastError();
  }));
  return HELM_OK;
}

// Dense variant: u (+)= (V (x) I) T^{-1} (V^T (x) I) x (3D: V_1 (x) V_2), with
// T the absorbing-boundary line matrices (sigma = lambda_A - w^2).
int dense_pass(helm_plan* p, int n, int64_t S, int64_t batch, const void* Q, const void* in, int in_kind,
               void* out, int out_kind, int accumulate, bool fp32, hipStream_t st) {
  DenseArgs g;
  g.n = n;
  g.S = S;
  g.batch = batch;
  g.Q = Q;
  g.in = in;
  g.in_kind = in_kind;
  g.out = out;
  g.out_kind = out_kind;
  g.accumulate = accumulate;
  g.skip = p->skip_cur;
  const double by = (double)batch * n * S * (esz_of(in_kind) + esz_of(out_kind) * (accumulate ? 2 : 1));
  HCHK(timed(p, K_DENSE, by, st, [&] { return launch_dense(g, fp32, st); }));
  return HELM_OK;
}

int solve_dense(helm_plan* p, const void* x, int x_kind, double2* u, int accumulate, int nb, bool fp32,
                hipStream_t st) {
  const int T = fp32 ? ST_C64 : ST_C128;
  void* W0 = p->W0.p;
  void* W1 = p->W1.p;
  const PAxis& A1 = p->ax[0];
  auto fwd = [&](const PAxis& A) { return fp32 ? A.Vf : A.Vd; };
  auto inv = [&](const PAxis& A) { return fp32 ? A.VTf : A.VTd; };
  LineArgs la;
  la.nb = nb;
  la.nL = p->nL;
  la.sC = make_double2(-p->cz, 0.0);
  la.hL = p->hL;
  la.kLo = p->kLo;
  la.kHi = p->kHi;
  la.skip = p->skip_cur;
  la.in_kind = T;
  la.out_kind = T;
  int rc;
  if (p->dim == 2) {
    const int n1 = A1.n, n2 = p->nL;
    rc = dense_pass(p, n1, n2, nb, fwd(A1), x, x_kind, W0, T, 0, fp32, st);
    if (rc) return rc;
    la.nO = 1;
    la.nI = n1;
    la.sTab = p->sig[1];
    la.piv = p->seed[1];
    la.in = W0;
    la.out = W0;
    la.tile = 0;
    tiles_for(p, 0, nb, 1, n1, n2, &la.tile, &la.ntiles);
    HCHK(timed(p, K_LINES, (double)nb * n1 * n2 * 2 * esz_of(T), st, [&] { return launch_lines(la, st); }));
    return dense_pass(p, n1, n2, nb, inv(A1), W0, T, u, ST_C128, accumulate, fp32, st);
  }
  const PAxis& A2 = p->ax[1];
  const int n1 = A1.n, n2 = A2.n, n3 = p->nL;
  rc = dense_pass(p, n1, (int64_t)n2 * n3, nb, fwd(A1), x, x_kind, W0, T, 0, fp32, st);
  if (rc) return rc;
  rc = dense_pass(p, n2, n3, (int64_t)nb * n1, fwd(A2), W0, T, W1, T, 0, fp32, st);
  if (rc) return rc;
  la.nO = n1;
  la.nI = n2;
  la.sTab = p->sig[3];
  la.piv = p->seed[3];
  la.in = W1;
  la.out = W1;
  tiles_for(p, 0, nb, n1, n2, n3, &la.tile, &la.ntiles);
  HCHK(timed(p, K_LINES, (double)nb * n1 * n2 * n3 * 2 * esz_of(T), st, [&] { return launch_lines(la, st); }));
  rc = dense_pass(p, n2, n3, (int64_t)nb * n1, inv(A2), W1, T, W0, T, 0, fp32, st);
  if (rc) return rc;
  return dense_pass(p, n1, (int64_t)n2 * n3, nb, inv(A1), W0, T, u, ST_C128, accumulate, fp32, st);
}

// Full solve of one precision pass: u (+)= A^{-1} x.
int solve_once(helm_plan* p, const void* x, int x_kind, double2* u, int accumulate, int nb, bool fp32,
               hipStream_t st) {
  if (p->dense) return solve_dense(p, x, x_kind, u, accumulate, nb, fp32, st);
  const int T = fp32 ? ST_C64 : ST_C128;
  const double w2 = p->cz;
  void* W0 = p->W0.p;
  void* W1 = p->W1.p;
  if (p->dim == 2) {
    const PAxis& A1 = p->ax[0];
    const int n1 = A1.n, n2 = p->nL;
    int rc = run_fft(p, A1, -1, fp32, x, x_kind, W0, T, nb, n2, A1.invmu, 1.0, 0, W1, T, st);
    if (rc) return rc;
    Level lv{nb, 1, n1, n2, &A1, w2};
    InnerIO io;
    io.in = W0;
    io.in_kind = T;
    io.out = W0;
    io.out_kind = T;
    io.seedB = p->seed[0];
    io.seedA = p->seed[1];
    io.sigTB = p->sig[0];
    io.sigTA = p->sig[1];
    rc = inner_solve(p, lv, io, st);
    if (rc) return rc;
    return run_fft(p, A1, +1, fp32, W0, T, u, ST_C128, nb, n2, nullptr, 1.0 / n1, accumulate, W1, T, st);
  }
  // 3D
  const PAxis& A1 = p->ax[0];
  const PAxis& A2 = p->ax[1];
  const int n1 = A1.n, n2 = A2.n, n3 = p->nL;
  const int64_t plane = (int64_t)n2 * n3;
  void* W2 = p->W2.p ? p->W2.p : W1;
  int rc = run_fft(p, A1, -1, fp32, x, x_kind, W1, T, nb, plane, A1.invmu, 1.0, 0, W2, T, st);
  if (rc) return rc;
  rc = run_fft(p, A2, -1, fp32, W1, T, W0, T, (int64_t)nb * n1, n3, A2.invmu, 1.0, 0, W2 == W1 ? W0 : W2, T, st);
  if (rc) return rc;
  Level lv{nb, n1, n2, n3, &A2, w2};
  double2* Vh = p->P0.as<double2>();  // [nb][2][n2][n3] scratch planes
  double2* Vp = p->P1.as<double2>();
  double2* Wp = p->P2.as<double2>();
  double2* Rh = p->P3.as<double2>();
  const double2* d_null = nullptr;
  (void)d_null;
  // Boundary steps from the plan's tables for this many right-hand sides?
  const bool cap = p->cap_min_nb > 0 && nb >= p->cap_min_nb;
  // Outer step 1: v_b.
  {
    InnerIO io;
    io.capS2 = cap;
    io.sO = A1.sigB;
    io.seedB = p->seed[0];
    io.seedA = p->seed[1];
    io.sigTB = p->sig[0];
    io.sigTA = p->sig[1];
    io.in = W0;
    io.in_kind = T;
    io.rhoL0 = A1.redB0;
    io.rhoL1 = A1.redB1;
    rc = inner_solve(p, lv, io, st);
    if (rc) return rc;
    rc = sum_to_planes(p, lv, Vh, st);
    if (rc) return rc;
    rc = run_fft(p, A2, +1, false, Vh, ST_C128, Vp, ST_C128, (int64_t)nb * 2, n3, nullptr, 1.0 / n2, 0,
                 Wp, ST_C128, st);
    if (rc) return rc;
  }
  // Outer step 2: r = C_1 v_b, w_b.
  {
    OuterMidArgs om;
    om.skip = p->skip_cur;
    om.nb = nb;
    om.n2 = n2;
    om.n3 = n3;
    om.a = Vp;
    om.c = nullptr;
    om.r = Wp;
    om.d1 = A1.bd;
    om.w2 = w2;
    om.h2 = A2.h;
    om.h3 = p->hL;
    om.k2Lo = corner_h(A2.glo, A2.h);
    om.k2Hi = corner_h(A2.ghi, A2.h);
    om.k3Lo = p->kLo;
    om.k3Hi = p->kHi;
    HCHK(timed(p, K_OUTER_MID, (double)nb * 2 * plane * sizeof(double2) * 3, st, [&] { return launch_outer_mid(om, st); }));
    if (cap) {
      // w_b = sum_l V1b[:, l] A_l^{-1} g_l with the inner absorbing
      // eigenvectors: A_l^{-1} = (V2 (x) I) blockdiag_m T_lm^{-1} (V2^T (x) I),
      // so w_b = (V2 (x) I) H_m (V2^T (x) I) r with the table H of
      // sum_l V1b[k, l] V1b[k', l] T_lm^{-1} per inner mode m
      rc = dense_pass(p, n2, n3, (int64_t)nb * 2, A2.Vd, Wp, ST_C128, Rh, ST_C128, 0, false, st);
      if (rc) return rc;
      rc = cap_apply(p, p->capH0, p->capH1, nb, n2, Rh, 2 * plane, n3, plane, Vh, 2 * plane, n3, plane, st);
      if (rc) return rc;
      rc = dense_pass(p, n2, n3, (int64_t)nb * 2, A2.VTd, Vh, ST_C128, Wp, ST_C128, 0, false, st);
      if (rc) return rc;
    } else {
      rc = run_fft(p, A2, -1, false, Wp, ST_C128, Rh, ST_C128, (int64_t)nb * 2, n3, A2.invmu, 1.0, 0, Vh,
                   ST_C128, st);
      if (rc) return rc;
      InnerIO io;
      io.sO = A1.sigA;
      io.seedB = p->seed[2];
      io.seedA = p->seed[3];
      io.sigTB = p->sig[2];
      io.sigTA = p->sig[3];
      io.PO = Rh;
      io.alpha0 = A1.va0d;
      io.alpha1 = A1.va1d;
      io.rhoL0 = A1.va0d;
      io.rhoL1 = A1.va1d;
      rc = inner_solve(p, lv, io, st);
      if (rc) return rc;
      rc = sum_to_planes(p, lv, Vh, st);
      if (rc) return rc;
      rc = run_fft(p, A2, +1, false, Vh, ST_C128, Wp, ST_C128, (int64_t)nb * 2, n3, nullptr, 1.0 / n2, 0,
                   Rh, ST_C128, st);
      if (rc) return rc;
    }
    // q = C_1 (v_b + w_b), transformed along x_2 and scaled by 1/mu_2; stored
    // in the lines' storage type, as the rank-2 rows of the Step-3 lines
    om.a = Vp;
    om.c = Wp;
    om.r = Vh;
    HCHK(timed(p, K_OUTER_MID, (double)nb * 2 * plane * sizeof(double2) * 3, st, [&] { return launch_outer_mid(om, st); }));
    rc = run_fft(p, A2, -1, false, Vh, ST_C128, Rh, T, (int64_t)nb * 2, n3, A2.invmu, 1.0, 0, Wp, ST_C128, st);
    if (rc) return rc;
  }
  // Outer step 3: corrected periodic solve, stored, then inverse transforms.
  {
    InnerIO io;
    io.capS2 = cap;
    io.sO = A1.sigB;
    io.seedB = p->seed[0];
    io.seedA = p->seed[1];
    io.sigTB = p->sig[0];
    io.sigTA = p->sig[1];
    io.in = W0;
    io.in_kind = T;
    io.PO = Rh;
    io.PO_kind = T;
    io.alpha0 = A1.genB0;
    io.alpha1 = A1.genB1;
    io.out = W0;
    io.out_kind = T;
    rc = inner_solve(p, lv, io, st);
    if (rc) return rc;
  }
  rc = run_fft(p, A2, +1, fp32, W0, T, W1, T, (int64_t)nb * n1, n3, nullptr, 1.0 / n2, 0, W2 == W1 ? W0 : W2,
               T, st);
  if (rc) return rc;
  return run_fft(p, A1, +1, fp32, W1, T, u, ST_C128, nb, plane, nullptr, 1.0 / n1, accumulate, W2 == W1 ? W0 : W2,
                 T, st);
}

int64_t npoints(const helm_plan* p) {
  int64_t n = 1;
  for (int j = 0; j < p->dim; ++j) n *= p->grid[j];
  return n;
}

// Workspace buffers of a solve, in a fixed order (the order of
// workspace_bytes and of the no-allocation layout).
enum WsSlot { WS_W0, WS_W1, WS_W2, WS_R, WS_PART, WS_VB, WS_PIB, WS_P0, WS_P1, WS_P2, WS_P3, WS_SCR, WS_NORMS,
              WS_BT1, WS_CTL, WS_N };

std::array<DevMem*, WS_N> ws_bufs(helm_plan* p) {
  return {&p->W0, &p->W1, &p->W2, &p->R, &p->part, &p->VB, &p->PIb, &p->P0,
          &p->P1, &p->P2, &p->P3, &p->scratch, &p->norms, &p->BT1, &p->ctl};
}

// Addresses of every workspace buffer a captured solve refers to.
std::array<void*, WS_N> workspace_addrs(helm_plan* p) {
  std::array<void*, WS_N> a;
  const auto b = ws_bufs(p);
  for (int i = 0; i < WS_N; ++i) a[i] = b[i]->p;
  return a;
}

// Bytes of every workspace buffer a solve of nb right-hand sides needs (0:
// not used by this plan).
std::array<size_t, WS_N> workspace_bytes(const helm_plan* p, int nb, bool fp32, bool need_r) {
  std::array<size_t, WS_N> w{};
  const int64_t N = npoints(p);
  const size_t esz = fp32 ? sizeof(float2) : sizeof(double2);
  w[WS_W0] = (size_t)N * nb * esz;
  w[WS_W1] = (size_t)N * nb * esz;
  if (p->dim == 3 && (p->ax[0].na > 1 || p->ax[1].na > 1)) w[WS_W2] = (size_t)N * nb * esz;
  if (need_r) w[WS_R] = (size_t)N * nb * esz;
  // partial sums: max over the reductions used
  size_t pe = 0;
  if (p->dim == 2) {
    pe = part_elems(1, nb, 1, p->ax[0].n, p->nL);
  } else {
    pe = std::max(part_elems(1, nb, p->ax[0].n, p->ax[1].n, p->nL),
                  part_elems(2, nb, p->ax[0].n, p->ax[1].n, p->nL));
  }
  w[WS_PART] = pe * sizeof(double2);
  const int64_t nO = p->dim == 2 ? 1 : p->ax[0].n;
  w[WS_VB] = (size_t)nb * nO * 2 * p->nL * sizeof(double2);
  w[WS_PIB] = w[WS_VB];
  if (p->dim == 3) {
    const size_t pl = (size_t)nb * 2 * p->ax[1].n * p->nL * sizeof(double2);
    w[WS_P0] = w[WS_P1] = w[WS_P2] = w[WS_P3] = pl;
  }
  // Bluestein temporaries: the largest [O][M][S] of any transform that uses them
  size_t tmax = 0;
  if (p->dim == 2) {
    if (p->ax[0].blue) tmax = (size_t)nb * p->ax[0].M * p->nL;
  } else {
    if (p->ax[0].blue) tmax = std::max(tmax, (size_t)nb * p->ax[0].M * p->ax[1].n * p->nL);
    if (p->ax[1].blue) tmax = std::max(tmax, (size_t)nb * std::max(p->ax[0].n, 2) * p->ax[1].M * p->nL);
  }
  w[WS_BT1] = tmax * sizeof(double2);
  w[WS_SCR] = (size_t)residual_scratch_len(p->dim, p->grid, nb) * sizeof(double);
  w[WS_NORMS] = (size_t)nb * 2 * sizeof(double);
  w[WS_CTL] = 64;
  return w;
}

int ensure_workspace_impl(helm_plan* p, int nb, bool fp32, bool need_r);

// Grows the workspace for nb right-hand sides; raises the plan's workspace
// generation when any buffer moved.
int ensure_workspace(helm_plan* p, int nb, bool fp32, bool need_r) {
  const auto before = workspace_addrs(p);
  const int rc = ensure_workspace_impl(p, nb, fp32, need_r);
  if (workspace_addrs(p) != before) ++p->ws_gen;
  return rc;
}

int ensure_workspace_impl(helm_plan* p, int nb, bool fp32, bool need_r) {
  const auto w = workspace_bytes(p, nb, fp32, need_r);
  const auto b = ws_bufs(p);
  for (int i = 0; i < WS_N; ++i)
    if (w[i]) HCHK(b[i]->ensure(w[i]));
  p->h_norms.resize(2 * nb);
  return HELM_OK;
}

ResidArgs resid_args(helm_plan* p, int nb) {
  ResidArgs a;
  a.skip = p->skip_cur;
  a.dim = p->dim;
  a.nb = nb;
  for (int j = 0; j < p->dim; ++j) {
    a.ax[j].n = (int)p->grid[j];
    a.ax[j].h = p->h[j];
    a.ax[j].kLo = corner_h(p->glo[j], p->h[j]);
    a.ax[j].kHi = corner_h(p->ghi[j], p->h[j]);
  }
  a.w2 = p->cz;
  a.norms = p->norms.as<double>();
  a.scratch = p->scratch.as<double>();
  a.scratch_len = (int64_t)(p->scratch.bytes / sizeof(double));
  a.r = nullptr;
  a.r_kind = ST_C128;
  return a;
}

// Residual norms -> host; returns max relative residual (NaN if non-finite).
int residual_norms(helm_plan* p, const double2* u, const double2* f, void* r, int r_kind, int nb,
                   hipStream_t st, double* relmax, std::vector<double>* rel) {
  ResidArgs a = resid_args(p, nb);
  a.u = u;
  a.f = f;
  a.r = r;
  a.r_kind = r_kind;
  HCHK(timed(p, K_RESID, (double)npoints(p) * nb * (2 * sizeof(double2) + (r ? esz_of(r_kind) : 0)), st,
             [&] { return launch_residual(a, st); }));
  double* hn = p->no_alloc ? p->h_norms_pin : p->h_norms.data();
  HCHK(hipMemcpyAsync(hn, a.norms, nb * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HCHK(hipStreamSynchronize(st));
  double mx = 0.0;
  if (rel) rel->assign(nb, 0.0);
  for (int b = 0; b < nb; ++b) {
    const double rr = hn[2 * b], ff = hn[2 * b + 1];
    if (!std::isfinite(rr) || !std::isfinite(ff)) {
      *relmax = NAN;
      return HELM_ENONFINITE;
    }
    const double v = ff > 0 ? std::sqrt(rr / ff) : 0.0;
    if (rel) (*rel)[b] = v;
    mx = std::max(mx, v);
  }
  *relmax = mx;
  return HELM_OK;
}

// Upload V[i][l] = v_l(i) and V^T, interleaved complex, in double and float.
// The four eigenvector arrays of an axis (V, V^T in double, then in float),
// for the device eigen-setup to fill.
int eigvec_buffers(PAxis& a, EigVecOut* o) {
  const size_t nn = (size_t)a.n * a.n;
  const size_t bd = 2 * nn * sizeof(double2), bf = 2 * nn * sizeof(float2);
  if (a.vmat.ensure(bd + bf) != hipSuccess) return HELM_ENOMEM;
  double2* d = a.vmat.as<double2>();
  float2* f = reinterpret_cast<float2*>((char*)a.vmat.p + bd);
  a.Vd = d;
  a.VTd = d + nn;
  a.Vf = f;
  a.VTf = f + nn;
  *o = EigVecOut{d, d + nn, f, f + nn};
  return HELM_OK;
}

int upload_eigvecs(PAxis& a, const std::vector<cd>& v) {
  const size_t n = (size_t)a.n, nn = n * n;
  std::vector<double2> hd(2 * nn);
  std::vector<float2> hf(2 * nn);
  for (size_t i = 0; i < n; ++i)
    for (size_t l = 0; l < n; ++l) {
      const cd x = v[i * n + l];
      hd[i * n + l] = make_double2(x.real(), x.imag());
      hd[nn + l * n + i] = make_double2(x.real(), x.imag());
    }
  for (size_t k = 0; k < 2 * nn; ++k) hf[k] = make_float2((float)hd[k].x, (float)hd[k].y);
  const size_t bd = 2 * nn * sizeof(double2), bf = 2 * nn * sizeof(float2);
  if (a.vmat.ensure(bd + bf) != hipSuccess) return HELM_ENOMEM;
  if (upload(a.vmat.p, hd.data(), bd) != hipSuccess) return HELM_EDEVICE;
  if (upload((char*)a.vmat.p + bd, hf.data(), bf) != hipSuccess) return HELM_EDEVICE;
  const double2* d = a.vmat.as<double2>();
  const float2* f = reinterpret_cast<const float2*>((char*)a.vmat.p + bd);
  a.Vd = d;
  a.VTd = d + nn;
  a.Vf = f;
  a.VTf = f + nn;
  return HELM_OK;
}

void fill_axis_tables_host(PAxis& a, long double czx, std::vector<double2>& buf, std::vector<double>& invmu) {
  const int n = a.n;
  const double h = a.h;
  buf.assign((size_t)n * 8, make_double2(0, 0));
  invmu.assign(n, 0.0);
  a.lamBx.assign(n, 0.0L);
  for (int l = 0; l < n; ++l) {
    const double th = 2.0 * M_PI * l / n;
    const double sh = std::sin(0.5 * th);
    const double omc = 2.0 * sh * sh;  // 1 - cos(theta) without cancellation
    const double cth = 1.0 - omc;
    const double mu = h / 6.0 * (4.0 + 2.0 * cth);
    const long double w2x = czx;
    const long double thx = 2.0L * (long double)M_PI * l / n;
    const long double shx = std::sin(0.5L * thx);
    const long double omcx = 2.0L * shx * shx;
    const long double lamBx = 6.0L * omcx / ((long double)h * (long double)h * (3.0L - omcx));
    a.lamBx[l] = lamBx;
    const double c = std::cos(th), s = std::sin(th);
    buf[0 * n + l] = make_double2((double)(lamBx - w2x), 0.0);             // sigB = lambda_B - w^2
    buf[1 * n + l] = make_double2((double)(a.lamAx[l].real() - w2x),       // sigA = lambda_A - w^2
                                  (double)a.lamAx[l].imag());
    buf[2 * n + l] = make_double2(1.0 / mu, 0.0);                          // genB0
    buf[3 * n + l] = make_double2(c / mu, s / mu);                         // genB1 = e^{+i th}/mu
    buf[4 * n + l] = make_double2(1.0 / n, 0.0);                           // redB0
    buf[5 * n + l] = make_double2(c / n, -s / n);                          // redB1 = e^{-i th}/n
    buf[6 * n + l] = hd2(a.va0[l]);
    buf[7 * n + l] = hd2(a.va1[l]);
    invmu[l] = 1.0 / mu;
  }
  // B - A on the two end nodes of this axis: the periodic corner 2/h against
  // the face's 1/h + g
  a.bd.dK[0][0] = make_double2(1.0 / h - a.glo.x, -a.glo.y);
  a.bd.dK[1][1] = make_double2(1.0 / h - a.ghi.x, -a.ghi.y);
  a.bd.dK[0][1] = a.bd.dK[1][0] = make_double2(-1.0 / h, 0.0);
  a.bd.dM[0][0] = a.bd.dM[1][1] = 2.0 * h / 6.0;
  a.bd.dM[0][1] = a.bd.dM[1][0] = h / 6.0;
}


// ---------------------------------------------------------------------------
// Refinement controlled on the device, for solves captured in a graph: the
// host cannot inspect residual norms between the steps, so a one-thread
// kernel evaluates them and raises a flag that turns every later launch of
// the same problem into an immediate return.
// ---------------------------------------------------------------------------
struct IrCtl {
  int done;        // nonzero: converged or failed, later launches return at once
  int iters;       // refinement steps taken after the first solve
  int status;      // HELM_* of the solve
  int pad;
  double rel_first;
  double rel_last;
};

__global__ void ir_reset_kernel(IrCtl* c, int done, IrCtl* mirror) {
  c->done = done;
  c->iters = 0;
  c->status = HELM_OK;
  c->pad = 0;
  c->rel_first = -1.0;
  c->rel_last = -1.0;
  if (mirror) *mirror = *c;
}

// After the residual of stage k (k = 0: first solve): converged, failed or
// one more refinement step.  Same rule as the host loop of helm_solve: stop
// at tol, at max_iter steps, or when a step fails to halve the residual.
__device__ void ir_update(const double* norms, int nb, double tol, int max_steps, int stage, IrCtl* c) {
  double mx = 0.0;
  bool bad = false;
  for (int b = 0; b < nb; ++b) {
    const double rr = norms[2 * b], ff = norms[2 * b + 1];
    if (!isfinite(rr) || !isfinite(ff)) bad = true;
    const double v = ff > 0.0 ? sqrt(rr / ff) : 0.0;
    mx = fmax(mx, v);
  }
  if (bad) {
    c->status = HELM_ENONFINITE;
    c->rel_last = NAN;
    c->done = 1;
    return;
  }
  const double prev = c->rel_last;
  if (stage == 0) c->rel_first = mx;
  c->rel_last = mx;
  if (mx <= tol) {
    c->status = HELM_OK;
    c->done = 1;
  } else if (stage >= max_steps || (stage > 0 && !(mx < 0.5 * prev))) {
    c->status = HELM_ENOCONV;
    c->done = 1;
  } else {
    c->iters = stage + 1;
  }
}

// With `mirror` set, the resulting state is also written there (pinned host
// memory that the host reads after the stream has drained).
__global__ void ir_check_kernel(const double* norms, int nb, double tol, int max_steps, int stage, IrCtl* c,
                                IrCtl* mirror) {
  if (!c->done) ir_update(norms, nb, tol, max_steps, stage, c);
  if (mirror) *mirror = *c;
}

// Enqueue one problem's complete solve with `steps` refinement steps whose
// launches are skipped on the device once the residual criterion is met.
// `limit` is the step count at which the check declares non-convergence:
// `steps` when the enqueued steps are all there will be, the plan's max_iter
// when the host may continue after them (the control block is then left
// not done).  Nothing here allocates or synchronises (the workspace must be
// in place).
int enqueue_device_ir(helm_plan* p, const double2* F, double2* U, int nb, int steps, int limit, IrCtl* mirror,
                      hipStream_t st) {
  const bool mixed = p->opt.precision == HELM_PREC_MIXED;
  const bool check = mixed || p->opt.check;
  IrCtl* c = p->ctl.as<IrCtl>();
  const bool prof = p->prof;
  p->prof = false;
  p->skip_cur = nullptr;
  int rc = HELM_OK;
  do {
    hipLaunchKernelGGL(ir_reset_kernel, dim3(1), dim3(1), 0, st, c, check ? 0 : 1, mirror);
    if (hipGetLastError() != hipSuccess) { rc = HELM_EDEVICE; break; }
    rc = solve_once(p, F, ST_C128, U, 0, nb, mixed, st);
    if (rc || !check) break;
    const int rk = mixed ? ST_C64 : ST_C128;
    for (int k = 0; k <= steps && !rc; ++k) {
      if (k > 0) {
        p->skip_cur = &c->done;
        rc = solve_once(p, p->R.p, rk, U, 1, nb, mixed, st);
        if (rc) break;
      }
      // the residual itself is the right-hand side of the next step; after
      // the last enqueued step only its norm is needed
      ResidArgs a = resid_args(p, nb);
      a.u = U;
      a.f = F;
      a.r = k < steps ? p->R.p : nullptr;
      a.r_kind = rk;
      if (launch_residual(a, st) != hipSuccess) { rc = HELM_EDEVICE; break; }
      hipLaunchKernelGGL(ir_check_kernel, dim3(1), dim3(1), 0, st, (const double*)a.norms, nb, p->opt.tol,
                         limit, k, c, mirror);
      if (hipGetLastError() != hipSuccess) rc = HELM_EDEVICE;
    }
  } while (false);
  p->skip_cur = nullptr;
  p->prof = prof;
  return rc;
}

// Capture the whole solve of (F, U, nb) with `steps` device-controlled
// refinement steps into the plan's graph.  The capture runs on an internal
// stream (the legacy default stream cannot be captured); the graph is
// launched on the caller's stream.
int capture_solve(helm_plan* p, const double2* F, double2* U, int nb, hipStream_t st, int steps) {
  p->drop_graph();
  if (!p->gcap && hipStreamCreateWithFlags(&p->gcap, hipStreamNonBlocking) != hipSuccess) return HELM_EDEVICE;
  if (!p->ctl_host && hipHostMalloc(&p->ctl_host, sizeof(IrCtl), hipHostMallocDefault) != hipSuccess) {
    p->ctl_host = nullptr;
    return HELM_ENOMEM;
  }
  if (hipStreamBeginCapture(p->gcap, hipStreamCaptureModeRelaxed) != hipSuccess) return HELM_EDEVICE;
  const int rc = enqueue_device_ir(p, F, U, nb, steps, p->opt.max_iter, static_cast<IrCtl*>(p->ctl_host), p->gcap);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(p->gcap, &g);
  if (rc || ce != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc ? rc : HELM_EDEVICE;
  }
  p->graph = g;
  if (hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    p->drop_graph();
    (void)hipGetLastError();
    return HELM_EDEVICE;
  }
  p->graph_key = helm_plan::Key{F, U, nb, st};
  p->graph_gen = p->ws_gen;
  p->graph_steps = steps;
  return HELM_OK;
}

// How the boundary steps of a solve of nrhs right-hand sides run.
int boundary_used(const helm_plan* p, int nrhs) {
  return (p->dim == 3 && !p->dense && p->cap_min_nb > 0 && nrhs >= p->cap_min_nb) ? HELM_BOUNDARY_TABLES
                                                                                   : HELM_BOUNDARY_LINES;
}

// Refinement on the host: while the residual exceeds tol, solve for the
// residual (stored in R by the last residual_norms) and add the correction
// to u; stop at tol, at max_iter steps, or when a step fails to halve the
// residual.  `it` steps were taken before, `rel` is the current residual.
// Fills the plan's report and returns its status.
int host_refine(helm_plan* p, const double2* F, double2* U, int nrhs, hipStream_t st, int it, double rel) {
  const bool mixed = p->opt.precision == HELM_PREC_MIXED;
  const int rk = mixed ? ST_C64 : ST_C128;
  helm_report& rep = p->rep;
  while (rel > p->opt.tol && it < p->opt.max_iter) {
    int rc = solve_once(p, p->R.p, rk, U, 1, nrhs, mixed, st);
    if (rc) return rep.status = rc;
    ++it;
    double nrel = 0;
    rc = residual_norms(p, U, F, p->R.p, rk, nrhs, st, &nrel, nullptr);
    rep.iterations = it;
    rep.rel_residual_max = nrel;
    if (rc) return rep.status = rc;
    if (!(nrel < 0.5 * rel)) {
      rel = nrel;
      break;  // stagnation
    }
    rel = nrel;
  }
  rep.iterations = it;
  rep.status = rel <= p->opt.tol ? HELM_OK : HELM_ENOCONV;
  return rep.status;
}

// helm_solve.  The first call with given arguments runs eagerly with the
// refinement loop on the host; a repeat of the same arguments (pointers,
// count, stream) captures the solve with as many device-controlled
// refinement steps as the previous call took and from then on launches the
// graph.  When the captured steps do not reach the tolerance, the host loop
// continues from the graph's last residual and the next call captures again
// with the larger count.  Profiling (per-kernel events) always runs eagerly.
int solve_entry(helm_plan* p, const void* f, void* u, int nrhs, hipStream_t st, bool allow_graph) {
  if (!p || !f || !u || nrhs < 1) return HELM_EINVAL;
  if (f == u) return HELM_EINVAL;
  const bool mixed = p->opt.precision == HELM_PREC_MIXED;
  const bool check = mixed || p->opt.check;
  helm_report& rep = p->rep;
  rep = helm_report{};
  rep.precision = p->opt.precision;
  rep.transform = p->dense ? HELM_TRANSFORM_DENSE : HELM_TRANSFORM_FFT;
  rep.boundary = boundary_used(p, nrhs);
  rep.nrhs = nrhs;
  rep.rel_residual_max = -1;
  rep.rel_residual_first = -1;
  int rc = ensure_workspace(p, nrhs, mixed, check);
  if (rc) return rep.status = rc;
  const double2* F = reinterpret_cast<const double2*>(f);
  double2* U = reinterpret_cast<double2*>(u);
  const int rk = mixed ? ST_C64 : ST_C128;
  const helm_plan::Key key{f, u, nrhs, st};
  const bool repeat = key == p->last_key;
  const int prev = p->prev_steps;
  p->last_key = key;
  p->prev_steps = -1;  // set again when this call completes
  int it = 0;
  double rel = 0;
  bool graph_ran = false;
  if (allow_graph && !p->prof) {
    if (p->graph_exec && !(p->graph_key == key && p->graph_gen == p->ws_gen)) p->drop_graph();
    if (!p->graph_exec && repeat && prev >= 0) {
      rc = capture_solve(p, F, U, nrhs, st, prev);
      if (rc) return rep.status = rc;
    }
    if (p->graph_exec) {
      if (hipGraphLaunch(p->graph_exec, st) != hipSuccess) return rep.status = HELM_EDEVICE;
      if (!check) {
        p->prev_steps = 0;
        return rep.status = HELM_OK;
      }
      if (hipStreamSynchronize(st) != hipSuccess) return rep.status = HELM_EDEVICE;
      IrCtl c;
      std::memcpy(&c, p->ctl_host, sizeof(IrCtl));
      graph_ran = true;
      rep.rel_residual_first = (c.status == HELM_ENONFINITE && c.rel_first < 0) ? NAN : c.rel_first;
      rep.rel_residual_max = c.rel_last;
      if (c.done) {
        rep.iterations = c.iters;
        p->prev_steps = c.iters;
        return rep.status = c.status;
      }
      // the captured steps were not enough: the host loop continues (the
      // last captured residual kept only its norm, so it is formed again);
      // the next call captures again
      it = p->graph_steps;
      rep.iterations = it;
      p->drop_graph();
      rc = residual_norms(p, U, F, p->R.p, rk, nrhs, st, &rel, nullptr);
      rep.rel_residual_max = rel;
      if (rc) return rep.status = rc;
    }
  }
  if (!graph_ran) {
    rc = solve_once(p, f, ST_C128, U, 0, nrhs, mixed, st);
    if (rc) return rep.status = rc;
    if (!check) {
      p->prev_steps = 0;
      return rep.status = HELM_OK;
    }
    rc = residual_norms(p, U, F, p->R.p, rk, nrhs, st, &rel, nullptr);
    rep.rel_residual_first = rel;
    rep.rel_residual_max = rel;
    if (rc) return rep.status = rc;
  }
  rc = host_refine(p, F, U, nrhs, st, it, rel);
  if (rc == HELM_OK || rc == HELM_ENOCONV) p->prev_steps = p->rep.iterations;
  return rc;
}

}  // namespace

}  // namespace helm

// ---------------------------------------------------------------------------
// Solves that allocate nothing (helm_solve_static).  Their workspace is this
// file-scope device array: every GPU the library runs on holds its own copy
// until the process ends.  In host code the name `scratch` is only a host-side
// stand-in; the device address is obtained once per device with
// hipGetSymbolAddress (static_workspace) and only that address is used.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[HELM_STATIC_SCRATCH_BYTES];

namespace helm {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch` (the device must be current).
int static_workspace(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return HELM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return HELM_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HELM_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// The plan's workspace buffers pointed into the static array for the scope
// of one solve, then restored (the plan's own buffers and captured graphs
// are untouched).
struct StaticWorkspace {
  helm_plan* p;
  std::array<std::pair<void*, size_t>, WS_N> saved;
  bool prof;
  StaticWorkspace(helm_plan* pl, const std::array<size_t, WS_N>& w) : p(pl) {
    const auto b = ws_bufs(p);
    char* base = static_cast<char*>(p->static_ws);
    size_t off = 0;
    for (int i = 0; i < WS_N; ++i) {
      saved[i] = {b[i]->p, b[i]->bytes};
      b[i]->p = w[i] ? base + off : nullptr;
      b[i]->bytes = w[i];
      off += round256(w[i]);
    }
    prof = p->prof;
    p->prof = false;  // per-kernel events would be created on first use
    p->no_alloc = true;
    p->skip_cur = nullptr;
  }
  ~StaticWorkspace() {
    const auto b = ws_bufs(p);
    for (int i = 0; i < WS_N; ++i) {
      b[i]->p = saved[i].first;
      b[i]->bytes = saved[i].second;
    }
    p->prof = prof;
    p->no_alloc = false;
  }
};

int solve_static(helm_plan* p, const void* f, void* u, int nrhs, hipStream_t st) {
  if (!p || !f || !u || nrhs < 1 || f == u) return HELM_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HELM_EDEVICE;
  if (dev != p->device || !p->static_ws || !p->h_norms_pin) return HELM_EINVAL;
  const bool mixed = p->opt.precision == HELM_PREC_MIXED;
  const bool check = mixed || p->opt.check;
  helm_report& rep = p->rep;
  rep = helm_report{};
  rep.precision = p->opt.precision;
  rep.transform = p->dense ? HELM_TRANSFORM_DENSE : HELM_TRANSFORM_FFT;
  rep.boundary = boundary_used(p, nrhs);
  rep.nrhs = nrhs;
  rep.rel_residual_max = -1;
  rep.rel_residual_first = -1;
  if (nrhs > HELM_STATIC_MAX_RHS) return rep.status = HELM_ENOMEM;
  const auto w = workspace_bytes(p, nrhs, mixed, check);
  size_t total = 0;
  for (size_t b : w) total += round256(b);
  if (total > (size_t)HELM_STATIC_SCRATCH_BYTES) return rep.status = HELM_ENOMEM;
  StaticWorkspace ws(p, w);
  const double2* F = reinterpret_cast<const double2*>(f);
  double2* U = reinterpret_cast<double2*>(u);
  int rc = solve_once(p, f, ST_C128, U, 0, nrhs, mixed, st);
  if (rc) return rep.status = rc;
  if (!check) return rep.status = HELM_OK;
  double rel = 0;
  rc = residual_norms(p, U, F, p->R.p, mixed ? ST_C64 : ST_C128, nrhs, st, &rel, nullptr);
  rep.rel_residual_first = rel;
  rep.rel_residual_max = rel;
  if (rc) return rep.status = rc;
  return host_refine(p, F, U, nrhs, st, 0, rel);
}

}  // namespace

}  // namespace helm

using namespace helm;

// ---------------------------------------------------------------------------
// Autotuner for the periodised-axis transform: times one solve of each
// variant on the plan's own shape and precision (one right-hand side, after a
// warm-up, best of three, HIP events) and keeps the faster.  Decisions can be
// cached in a text file, one line per shape:
//   helm-tune dim=<d> grid=<n1>x<n2>x<n3> prec=<p> transform=<t> fft_ms=<..> dense_ms=<..>
// ---------------------------------------------------------------------------
std::string tune_key(const helm_plan* p) {
  char buf[160];
  std::snprintf(buf, sizeof buf, "dim=%d grid=%lldx%lldx%lld prec=%d", p->dim, (long long)p->grid[0],
                (long long)p->grid[1], (long long)(p->dim == 3 ? p->grid[2] : 1), p->opt.precision);
  return buf;
}

// Value of `field` (e.g. "transform=") on the last cache line for this key.
bool tune_lookup(const std::string& path, const std::string& key, const char* field, int* value) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  const std::string pre = "helm-tune " + key + " " + field;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    if (std::strncmp(line, pre.c_str(), pre.size()) != 0) continue;
    *value = std::atoi(line + pre.size());
    found = true;  // the last matching line wins
  }
  std::fclose(f);
  return found;
}

bool tune_lookup(const std::string& path, const std::string& key, int* choice) {
  int t = 0;
  if (!tune_lookup(path, key, "transform=", &t)) return false;
  if (t != HELM_TRANSFORM_FFT && t != HELM_TRANSFORM_DENSE) return false;
  *choice = t;
  return true;
}

// ---------------------------------------------------------------------------
// Boundary operator tables (3D).  W_l^{kk'} = sum_m V2b[k,m] V2b[k',m]
// (T^{BA}_lm)^{-1} maps the inner boundary vectors to the inner Step-2
// result of outer mode l; H_m^{kk'} = sum_l V1b[k,l] V1b[k',l] (T^{AA}_lm)^{-1}
// maps the inner absorbing mode m of the outer boundary planes to that of the
// outer Step-2 result.  Column x' of each is the reduction of the line
// solutions with the unit right-hand side e_{x'}: one line launch per k'
// with nL "right-hand sides".
// ---------------------------------------------------------------------------
int build_boundary_tables(helm_plan* p) {
  const PAxis& A1 = p->ax[0];
  const PAxis& A2 = p->ax[1];
  const int n1 = A1.n, n2 = A2.n, nL = p->nL;
  std::vector<double2> w((size_t)3 * (n1 + n2));
  for (int m = 0; m < n2; ++m) {
    w[m] = hd2(A2.va0[m] * A2.va0[m]);
    w[n2 + m] = hd2(A2.va0[m] * A2.va1[m]);
    w[2 * n2 + m] = hd2(A2.va1[m] * A2.va1[m]);
  }
  double2* d1 = w.data() + 3 * n2;
  for (int l = 0; l < n1; ++l) {
    d1[l] = hd2(A1.va0[l] * A1.va0[l]);
    d1[n1 + l] = hd2(A1.va0[l] * A1.va1[l]);
    d1[2 * n1 + l] = hd2(A1.va1[l] * A1.va1[l]);
  }
  DevMem wt;
  HCHK(wt.ensure(w.size() * sizeof(double2)));
  HCHK(upload(wt.p, w.data(), w.size() * sizeof(double2)));
  const double2* c = wt.as<double2>();        // c00, c01, c11 over m
  const double2* dd = c + 3 * (size_t)n2;     // d00, d01, d11 over l
  const size_t blkW = (size_t)nL * n1 * 2 * nL, blkH = (size_t)nL * n2 * 2 * nL;
  const size_t esz = p->cap_fp32 ? sizeof(float2) : sizeof(double2);
  HCHK(p->capW.ensure(2 * blkW * esz));
  HCHK(p->capH.ensure(2 * blkH * esz));
  p->capW0 = p->capW.p;
  p->capW1 = static_cast<char*>(p->capW.p) + blkW * esz;
  p->capH0 = p->capH.p;
  p->capH1 = static_cast<char*>(p->capH.p) + blkH * esz;
  DevMem part, stage;  // line partials; one table block in the reductions' layout
  HCHK(part.ensure(std::max(part_elems(1, nL, n1, n2, nL), part_elems(2, nL, n1, n2, nL)) * sizeof(double2)));
  HCHK(stage.ensure(std::max(blkW, blkH) * sizeof(double2)));
  LineArgs base;
  base.nb = nL;
  base.nO = n1;
  base.nI = n2;
  base.nL = nL;
  base.hL = p->hL;
  base.kLo = p->kLo;
  base.kHi = p->kHi;
  base.unit_rhs = 1;
  base.part = part.as<double2>();
  for (int kp = 0; kp < 2; ++kp) {
    LineArgs la = base;  // W: lines of the (B, A) family, reduced over m
    la.sTab = p->sig[1];
    la.piv = p->seed[1];
    la.red = 1;
    la.rho0 = kp ? c + n2 : c;
    la.rho1 = kp ? c + 2 * n2 : c + n2;
    tiles_for(p, 1, nL, n1, n2, nL, &la.tile, &la.ntiles);
    HCHK(launch_lines(la, nullptr));
    HCHK(launch_sum_partials(base.part, nL * n1, la.ntiles, nL, stage.as<double2>(), nullptr, nullptr));
    HCHK(launch_cap_reorder(stage.as<double2>(), const_cast<void*>(kp ? p->capW1 : p->capW0), n1, nL,
                            p->cap_fp32 != 0, nullptr));
  }
  for (int kp = 0; kp < 2; ++kp) {
    LineArgs la = base;  // H: lines of the (A, A) family, reduced over l
    la.sTab = p->sig[3];
    la.piv = p->seed[3];
    la.red = red_l_mode(p);
    la.rho0 = kp ? dd + n1 : dd;
    la.rho1 = kp ? dd + 2 * n1 : dd + n1;
    tiles_for(p, 2, nL, n1, n2, nL, &la.tile, &la.ntiles);
    HCHK(launch_lines(la, nullptr));
    HCHK(launch_sum_partials(base.part, nL * n2, la.ntiles, nL, stage.as<double2>(), nullptr, nullptr));
    HCHK(launch_cap_reorder(stage.as<double2>(), const_cast<void*>(kp ? p->capH1 : p->capH0), n2, nL,
                            p->cap_fp32 != 0, nullptr));
  }
  HCHK(hipDeviceSynchronize());
  return HELM_OK;
}

// Times (ms, best of 3 after a warm-up) of the boundary work of one 3D solve
// of nb right-hand sides that the tables replace: 5 Step-2-like line sweeps
// (measured as one sweep times 5) against two capW products, one capH
// product and the two inner eigenvector transforms of the boundary planes.
int measure_boundary(helm_plan* p, int nb, double* t_lines, double* t_tab) {
  const PAxis& A2 = p->ax[1];
  const int n1 = p->ax[0].n, n2 = A2.n, nL = p->nL;
  const int64_t per = 2 * (int64_t)nL, plane = (int64_t)n2 * nL;
  DevMem pi, part, pa, pb;
  HCHK(pi.ensure((size_t)nb * n1 * per * sizeof(double2)));
  HCHK(part.ensure(part_elems(1, nb, n1, n2, nL) * sizeof(double2)));
  HCHK(pa.ensure((size_t)nb * 2 * plane * sizeof(double2)));
  HCHK(pb.ensure((size_t)nb * 2 * plane * sizeof(double2)));
  HCHK(hipMemset(pi.p, 0x3f, pi.bytes));  // finite values of order 1e-3
  HCHK(hipMemset(pa.p, 0x3f, pa.bytes));
  LineArgs s2;
  s2.nb = nb;
  s2.nO = n1;
  s2.nI = n2;
  s2.nL = nL;
  s2.hL = p->hL;
  s2.kLo = p->kLo;
  s2.kHi = p->kHi;
  s2.sTab = p->sig[1];
  s2.piv = p->seed[1];
  s2.PI = pi.p;
  s2.r2_kind = ST_C128;
  s2.beta0 = A2.va0d;
  s2.beta1 = A2.va1d;
  s2.red = 1;
  s2.rho0 = A2.va0d;
  s2.rho1 = A2.va1d;
  s2.part = part.as<double2>();
  tiles_for(p, 1, nb, n1, n2, nL, &s2.tile, &s2.ntiles);
  auto lines = [&]() -> int {
    HCHK(launch_lines(s2, nullptr));
    return HELM_OK;
  };
  auto tab = [&]() -> int {
    const int64_t gs = (int64_t)n1 * per;
    for (int k = 0; k < 2; ++k) {
      const int rc = cap_apply(p, p->capW0, p->capW1, nb, n1, pi.as<double2>(), gs, per, nL, part.as<double2>(),
                               gs, per, nL, nullptr);
      if (rc) return rc;
    }
    int rc = dense_pass(p, n2, nL, (int64_t)nb * 2, A2.Vd, pa.p, ST_C128, pb.p, ST_C128, 0, false, nullptr);
    if (rc) return rc;
    rc = cap_apply(p, p->capH0, p->capH1, nb, n2, pb.as<double2>(), 2 * plane, nL, plane, pa.as<double2>(),
                   2 * plane, nL, plane, nullptr);
    if (rc) return rc;
    return dense_pass(p, n2, nL, (int64_t)nb * 2, A2.VTd, pa.p, ST_C128, pb.p, ST_C128, 0, false, nullptr);
  };
  hipEvent_t e0, e1;
  HCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return HELM_EDEVICE;
  }
  int rc = HELM_OK;
  double best[2] = {1e30, 1e30};
  for (int which = 0; which < 2 && !rc; ++which) {
    for (int rep = 0; rep < 4 && !rc; ++rep) {
      if (hipEventRecord(e0, nullptr) != hipSuccess) { rc = HELM_EDEVICE; break; }
      rc = which == 0 ? lines() : tab();
      if (rc) break;
      float ms = 0;
      if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = HELM_EDEVICE;
        break;
      }
      if (rep > 0) best[which] = std::min(best[which], (double)ms);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *t_lines = 5.0 * best[0];
  *t_tab = best[1];
  return rc;
}

// Layout of the line reductions over the outer modes (3D): fixed by
// HELM_RED_L_LAYOUT (2 or 3) when set, else the cached decision, else the
// faster of the two on an outer-Step-1 sweep of one right-hand side (read of
// an N-sized input, generated rank-2 term, weighted sums over l; best of 3
// after a warm-up), appended to the cache.
int tune_layout(helm_plan* p) {
  const char* env = std::getenv("HELM_RED_L_LAYOUT");
  if (env && (env[0] == '2' || env[0] == '3') && env[1] == 0) {
    p->red_layout = env[0] - '0';
    return HELM_OK;
  }
  const std::string key = tune_key(p);
  int cached = 0;
  if (!p->tune_path.empty() && tune_lookup(p->tune_path, key, "layout=", &cached) && (cached == 2 || cached == 3)) {
    p->red_layout = cached;
    return HELM_OK;
  }
  const PAxis& A1 = p->ax[0];
  const PAxis& A2 = p->ax[1];
  const int n1 = A1.n, n2 = A2.n, nL = p->nL;
  const bool fp32 = p->opt.precision == HELM_PREC_MIXED;
  const size_t esz = fp32 ? sizeof(float2) : sizeof(double2);
  DevMem in, pi, part;
  HCHK(in.ensure((size_t)n1 * n2 * nL * esz));
  HCHK(pi.ensure((size_t)n1 * 2 * nL * sizeof(double2)));
  HCHK(part.ensure(part_elems(2, 1, n1, n2, nL) * sizeof(double2)));
  HCHK(hipMemset(in.p, 0x3f, in.bytes));  // finite values of order 1e-3 (1 in complex64)
  HCHK(hipMemset(pi.p, 0x3f, pi.bytes));
  LineArgs la;
  la.nb = 1;
  la.nO = n1;
  la.nI = n2;
  la.nL = nL;
  la.hL = p->hL;
  la.kLo = p->kLo;
  la.kHi = p->kHi;
  la.sTab = p->sig[0];
  la.piv = p->seed[0];
  la.in = in.p;
  la.in_kind = fp32 ? ST_C64 : ST_C128;
  la.PI = pi.p;  // in the storage type of the lines (filled with finite bytes either way)
  la.r2_kind = la.in_kind;
  la.beta0 = A2.genB0;
  la.beta1 = A2.genB1;
  la.rho0 = A1.redB0;
  la.rho1 = A1.redB1;
  la.part = part.as<double2>();
  hipEvent_t e0, e1;
  HCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return HELM_EDEVICE;
  }
  int rc = HELM_OK;
  double best[2] = {1e30, 1e30};
  for (int v = 0; v < 2 && !rc; ++v) {
    la.red = 2 + v;
    tiles_for_layout(2, la.red, 1, n1, n2, nL, &la.tile, &la.ntiles);
    for (int rep = 0; rep < 4 && !rc; ++rep) {
      float ms = 0;
      if (hipEventRecord(e0, nullptr) != hipSuccess || launch_lines(la, nullptr) != hipSuccess ||
          hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = HELM_EDEVICE;
        break;
      }
      if (rep > 0) best[v] = std::min(best[v], (double)ms);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  p->red_layout = best[1] < best[0] ? 3 : 2;
  if (!p->tune_path.empty()) {
    FILE* f = std::fopen(p->tune_path.c_str(), "a");
    if (f) {
      std::fprintf(f, "helm-tune %s layout=%d layout2_ms=%.6g layout3_ms=%.6g\n", key.c_str(), p->red_layout,
                   best[0], best[1]);
      std::fclose(f);
    }
  }
  return HELM_OK;
}

// Form of the 512-point transform passes (plans with such a pass along a
// power-of-two axis): the 128 KB tile with one block per tile, the 64 KB
// complex64 tile (two blocks per compute unit; mixed-precision plans only),
// or the streaming pass (one persistent block per compute unit, the next
// tile's loads in flight), each timed on the forward transform along the
// first such axis over a volume of the plan's shape and precision; cached as
// "fft512=".
int tune_fft_tile(helm_plan* p) {
  const bool fp32 = p->opt.precision == HELM_PREC_MIXED;
  int axis = -1;
  for (int j = 0; j < p->nper && axis < 0; ++j) {
    const PAxis& a = p->ax[j];
    // (chirp-z axes keep the default: their passes use the solve's workspace)
    const bool u512 = !a.blue && (a.n == 512 || a.na == 512 || a.nbp == 512);
    if (u512) axis = j;
  }
  if (axis < 0) return HELM_OK;
  // candidates: 0 the 128 KB tile, 1 the 64 KB complex64 tile, 2 the
  // streaming pass (128 KB tiles, next tile's loads in flight)
  const int nv = 3;
  const bool cand[3] = {true, fp32, true};
  const std::string key = tune_key(p);
  int cached = -1;
  if (!p->tune_path.empty() && tune_lookup(p->tune_path, key, "fft512=", &cached) && cached >= 0 && cached < nv &&
      cand[cached]) {
    p->fft_small = cached;
    return HELM_OK;
  }
  int64_t N = 1;
  for (int j = 0; j < p->dim; ++j) N *= p->grid[j];
  int64_t O = 1, S = 1;
  for (int j = 0; j < axis; ++j) O *= p->grid[j];
  for (int j = axis + 1; j < p->dim; ++j) S *= p->grid[j];
  const PAxis& A = p->ax[axis];
  const int T = fp32 ? ST_C64 : ST_C128;
  const size_t bytes = (size_t)N * (fp32 ? sizeof(float2) : sizeof(double2));
  DevMem in, out, tmp;
  HCHK(in.ensure(bytes));
  HCHK(out.ensure(bytes));
  HCHK(tmp.ensure(bytes));
  HCHK(hipMemset(in.p, 0x3c, in.bytes));  // finite values (order 1e-2 in FP32, 1e-18 in FP64)
  hipEvent_t e0, e1;
  HCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return HELM_EDEVICE;
  }
  int rc = HELM_OK;
  double best[3] = {1e30, 1e30, 1e30};
  for (int v = 0; v < nv && !rc; ++v) {
    if (!cand[v]) continue;
    p->fft_small = v;
    for (int rep = 0; rep < 4 && !rc; ++rep) {
      float ms = 0;
      if (hipEventRecord(e0, nullptr) != hipSuccess) rc = HELM_EDEVICE;
      if (!rc) rc = run_fft(p, A, -1, fp32, in.p, T, out.p, T, O, S, nullptr, 1.0, 0, tmp.p, T, nullptr);
      if (!rc && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = HELM_EDEVICE;
      if (!rc && rep > 0) best[v] = std::min(best[v], (double)ms);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  int pick = 0;
  for (int v = 1; v < nv; ++v)
    if (cand[v] && best[v] < best[pick]) pick = v;
  p->fft_small = pick;
  if (!p->tune_path.empty()) {
    FILE* f = std::fopen(p->tune_path.c_str(), "a");
    if (f) {
      std::fprintf(f, "helm-tune %s fft512=%d tile128k_ms=%.6g tile64k_ms=%.6g stream_ms=%.6g\n", key.c_str(), pick,
                   best[0], cand[1] ? best[1] : -1.0, best[2]);
      std::fclose(f);
    }
  }
  return HELM_OK;
}

// Chirp-z transforms (axes whose length is not a power of two): the
// convolution in two or three passes over the padded length M (row
// segments of up to 32 columns) or in one pass with the whole M-point
// transform in LDS (narrower tiles: 4 to 8 columns, but the padded rows
// never reach memory).  Timed per such axis on a volume of the plan's shape
// and precision; cached as "chirp<axis>=".
bool onepass_length(int M) {
  return M == 576 || M == 1152 || M == 2304 || M == 4608 || M == 1024 || M == 2048 ||
         (M >= 2 && M <= 512 && !(M & (M - 1)));
}

int tune_chirp(helm_plan* p) {
  const bool fp32 = p->opt.precision == HELM_PREC_MIXED;
  const int T = fp32 ? ST_C64 : ST_C128;
  const size_t esz = fp32 ? sizeof(float2) : sizeof(double2);
  const std::string key = tune_key(p);
  int64_t N = 1;
  for (int j = 0; j < p->dim; ++j) N *= p->grid[j];
  for (int j = 0; j < p->nper; ++j) {
    PAxis& A = p->ax[j];
    if (!A.blue || !onepass_length(A.M)) continue;
    char field[16];
    std::snprintf(field, sizeof field, "chirp%d=", j);
    int cached = -1;
    if (!p->tune_path.empty() && tune_lookup(p->tune_path, key, field, &cached) && (cached == 0 || cached == 1)) {
      A.onepass = cached;
      continue;
    }
    int64_t O = 1, S = 1;
    for (int i = 0; i < j; ++i) O *= p->grid[i];
    for (int i = j + 1; i < p->dim; ++i) S *= p->grid[i];
    DevMem in, out, t1;
    HCHK(in.ensure((size_t)N * esz));
    HCHK(out.ensure((size_t)N * esz));
    HCHK(t1.ensure((size_t)O * A.M * S * esz));
    HCHK(hipMemset(in.p, 0x3c, in.bytes));  // finite values
    // the multi-pass form takes its padded rows from the plan's chirp buffer
    std::swap(p->BT1.p, t1.p);
    std::swap(p->BT1.bytes, t1.bytes);
    hipEvent_t e0, e1;
    int rc = hipEventCreate(&e0) == hipSuccess ? HELM_OK : HELM_EDEVICE;
    if (!rc && hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      rc = HELM_EDEVICE;
    }
    double best[2] = {1e30, 1e30};
    if (!rc) {
      for (int v = 0; v < 2 && !rc; ++v) {
        A.onepass = v;
        for (int rep = 0; rep < 4 && !rc; ++rep) {
          float ms = 0;
          if (hipEventRecord(e0, nullptr) != hipSuccess) rc = HELM_EDEVICE;
          if (!rc) rc = run_fft(p, A, -1, fp32, in.p, T, out.p, T, O, S, nullptr, 1.0, 0, nullptr, T, nullptr);
          if (!rc && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                      hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = HELM_EDEVICE;
          if (!rc && rep > 0) best[v] = std::min(best[v], (double)ms);
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    std::swap(p->BT1.p, t1.p);
    std::swap(p->BT1.bytes, t1.bytes);
    if (rc) return rc;
    A.onepass = best[1] < best[0] ? 1 : 0;
    if (!p->tune_path.empty()) {
      FILE* f = std::fopen(p->tune_path.c_str(), "a");
      if (f) {
        std::fprintf(f, "helm-tune %s %s%d multipass_ms=%.6g onepass_ms=%.6g\n", key.c_str(), field, A.onepass,
                     best[0], best[1]);
        std::fclose(f);
      }
    }
  }
  return HELM_OK;
}

// Builds the tables when they fit the budget and decides from which number
// of right-hand sides solves use them (helm_options.boundary).
int setup_boundary_tables(helm_plan* p) {
  const bool forced = p->opt.boundary == HELM_BOUNDARY_TABLES;
  const int n1 = p->ax[0].n, n2 = p->ax[1].n, nL = p->nL;
  if ((int64_t)nL * n1 * n2 >= 0x7fffffffLL) return forced ? HELM_EUNSUPPORTED : HELM_OK;
  const double bytes = (p->opt.precision == HELM_PREC_MIXED ? 32.0 : 64.0) * nL * nL * (double)(n1 + n2);
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return HELM_EDEVICE;
  const double budget = std::min(32.0 * (double)(1ull << 30), 0.25 * (double)fr);
  if (!forced && bytes > budget) return HELM_OK;
  const std::string key = tune_key(p);
  int cached = -1;
  if (!forced && !p->tune_path.empty() && tune_lookup(p->tune_path, key, "boundary cap_min_nb=", &cached) &&
      cached == 0)
    return HELM_OK;  // measured before: the tables never pay for this shape
  // the mixed-precision path keeps its tables in complex64, like its other
  // bulk data (they are applied to FP64 boundary vectors with FP64 sums)
  p->cap_fp32 = p->opt.precision == HELM_PREC_MIXED;
  int rc = build_boundary_tables(p);
  if (rc) return rc;
  if (forced) {
    p->cap_min_nb = 1;
    return HELM_OK;
  }
  if (cached > 0) {
    p->cap_min_nb = cached;
    return HELM_OK;
  }
  // time both forms at 1 and 16 right-hand sides; both grow linearly with nb
  rc = measure_boundary(p, 1, &p->cap_ms[0], &p->cap_ms[2]);
  if (!rc) rc = measure_boundary(p, 16, &p->cap_ms[1], &p->cap_ms[3]);
  if (rc) return rc;
  const double bl = (p->cap_ms[1] - p->cap_ms[0]) / 15.0, al = p->cap_ms[0] - bl;
  const double bt = (p->cap_ms[3] - p->cap_ms[2]) / 15.0, at = p->cap_ms[2] - bt;
  int nmin = 0;
  if (p->cap_ms[2] < p->cap_ms[0]) {
    nmin = 1;
  } else if (bl > bt) {
    const double x = (at - al) / (bl - bt);  // tables win above x right-hand sides
    nmin = x < 1e6 ? (int)std::floor(x) + 1 : 0;
  }
  p->cap_min_nb = nmin;
  if (nmin == 0) {  // never pays: give the memory back
    p->capW.release();
    p->capH.release();
    p->capW0 = p->capW1 = p->capH0 = p->capH1 = nullptr;
  }
  if (!p->tune_path.empty()) {
    FILE* f = std::fopen(p->tune_path.c_str(), "a");
    if (f) {
      std::fprintf(f, "helm-tune %s boundary cap_min_nb=%d lines_ms_1=%.6g lines_ms_16=%.6g tables_ms_1=%.6g "
                   "tables_ms_16=%.6g\n", key.c_str(), nmin, p->cap_ms[0], p->cap_ms[1], p->cap_ms[2], p->cap_ms[3]);
      std::fclose(f);
    }
  }
  return HELM_OK;
}

int autotune_transform(helm_plan* p) {
  int choice = 0;
  const std::string key = tune_key(p);
  if (!p->tune_path.empty() && tune_lookup(p->tune_path, key, &choice)) {
    p->dense = choice == HELM_TRANSFORM_DENSE;
    return HELM_OK;
  }
  const bool fp32 = p->opt.precision == HELM_PREC_MIXED;
  const int wrc = ensure_workspace(p, 1, fp32, false);
  if (wrc != HELM_OK) return wrc;
  const int64_t N = npoints(p);
  DevMem tf, tu;
  HCHK(tf.ensure((size_t)N * sizeof(double2)));
  HCHK(tu.ensure((size_t)N * sizeof(double2)));
  HCHK(hipMemset(tf.p, 0x3f, (size_t)N * sizeof(double2)));  // finite values of order 1e-3
  hipEvent_t e0, e1;
  HCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return HELM_EDEVICE;
  }
  int rc = HELM_OK;
  const bool prof = p->prof;
  p->prof = false;
  for (int cand = 0; cand < 2 && !rc; ++cand) {
    p->dense = cand;
    float best = 1e30f;
    for (int rep = 0; rep < 4 && !rc; ++rep) {
      if (hipEventRecord(e0, nullptr) != hipSuccess) { rc = HELM_EDEVICE; break; }
      rc = solve_once(p, tf.p, ST_C128, tu.as<double2>(), 0, 1, fp32, nullptr);
      if (rc) break;
      if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = HELM_EDEVICE;
        break;
      }
      float ms = 0;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = HELM_EDEVICE; break; }
      if (rep > 0) best = std::min(best, ms);  // rep 0 is the warm-up
    }
    p->tune_ms[cand] = best;
  }
  p->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  p->dense = p->tune_ms[1] < p->tune_ms[0] ? 1 : 0;
  if (!p->tune_path.empty()) {
    FILE* f = std::fopen(p->tune_path.c_str(), "a");
    if (f) {
      std::fprintf(f, "helm-tune %s transform=%d fft_ms=%.6g dense_ms=%.6g\n", key.c_str(),
                   p->dense ? HELM_TRANSFORM_DENSE : HELM_TRANSFORM_FFT, p->tune_ms[0], p->tune_ms[1]);
      std::fclose(f);
    }
  }
  return HELM_OK;
}

// A batch of independent plans solved by one graph launch.  Each plan keeps
// its own workspace; the plans' pipelines are spread over side streams
// inside one stream capture (longest first onto the least loaded stream), so
// the graph has one independent branch per stream.
// Most parallel branches (side streams) of a batch graph.
constexpr int kBatchMaxBranches = 16;

struct helm_batch;
std::string batch_key(const helm_batch* b, const int* nrhs);

struct helm_batch {
  std::vector<helm_plan*> plans;
  int max_nrhs = 1;
  int device = 0;
  hipStream_t cap = nullptr;  // capture origin (the legacy default stream cannot be captured)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // inputs the current graph was captured for
  std::vector<const void*> kf;
  std::vector<void*> ku;
  std::vector<int> kn;
  std::vector<uint64_t> kgen;  // workspace generation of each plan at capture
  hipStream_t kst = nullptr;
  std::vector<int> steps;  // refinement steps captured per plan
  int branches = 0;        // parallel branches of the graph (side streams used), 0 = not chosen yet
  hipStream_t last = nullptr;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~helm_batch() {
    (void)hipDeviceSynchronize();
    drop_graph();
    for (auto s : side) (void)hipStreamDestroy(s);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
  }
};

// Tune-cache key of a batch: its size and a hash (FNV-1a) of every problem's
// shape, precision and number of right-hand sides.
std::string batch_key(const helm_batch* b, const int* nrhs) {
  uint64_t hsh = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int k = 0; k < 8; ++k) {
      hsh ^= (uint64_t)(v >> (8 * k)) & 0xff;
      hsh *= 1099511628211ull;
    }
  };
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const helm_plan* p = b->plans[i];
    mix(p->dim);
    for (int j = 0; j < p->dim; ++j) mix(p->grid[j]);
    mix(p->opt.precision);
    mix(nrhs[i]);
  }
  char buf[96];
  std::snprintf(buf, sizeof buf, "batch=%zu shapes=%016llx", b->plans.size(), (unsigned long long)hsh);
  return buf;
}

extern "C" {

void helm_default_options(helm_options* opt) {
  if (!opt) return;
  opt->precision = HELM_PREC_FP64;
  opt->tol = 1e-10;
  opt->max_iter = 8;
  opt->check = 1;
  opt->transform = HELM_TRANSFORM_FFT;
  opt->tune_cache = nullptr;
  opt->boundary = HELM_BOUNDARY_AUTO;
  opt->eigen = HELM_EIGEN_AUTO;
}

const char* helm_strerror(int code) {
  switch (code) {
    case HELM_OK: return "success";
    case HELM_EINVAL: return "invalid argument";
    case HELM_ENOMEM: return "out of memory";
    case HELM_EDEVICE: return "HIP device error";
    case HELM_ESINGULAR: return "singular system";
    case HELM_ENOCONV: return "refinement did not converge";
    case HELM_ENONFINITE: return "non-finite value in right-hand side or residual";
    case HELM_EUNSUPPORTED: return "unsupported problem for this build";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {

// Which coefficient sets the method handles (every line system and the
// operator nonsingular):
//  * c = 0 and g = 0 on every face: A annihilates the constants (ESINGULAR);
//  * some face of the last axis with Im g != 0, and no two faces with Im g
//    of opposite signs: with sigma real (periodic branch) the imaginary part
//    of v^H T v is sum Im g |v_face|^2, nonzero for a null vector of an
//    irreducible tridiagonal T, and the absorbing-branch sigma carry
//    imaginary parts of the same sign;
//  * all g real and >= 0, and c < 0, or c = 0 with g > 0 on a face of the
//    last axis: every line matrix sigma M + K is symmetric positive definite;
//  * otherwise (c > 0 with real faces on the last axis, mixed signs)
//    resonant line systems are possible: EUNSUPPORTED.
int check_coefficients(int dim, double c, const double2* glo, const double2* ghi) {
  if (!std::isfinite(c)) return HELM_EINVAL;
  bool all_zero = c == 0.0, all_real = true, neg_re = false, pos_im = false, neg_im = false;
  for (int j = 0; j < dim; ++j) {
    for (const double2 g : {glo[j], ghi[j]}) {
      if (!std::isfinite(g.x) || !std::isfinite(g.y)) return HELM_EINVAL;
      all_zero = all_zero && g.x == 0.0 && g.y == 0.0;
      all_real = all_real && g.y == 0.0;
      neg_re = neg_re || g.x < 0.0;
      pos_im = pos_im || g.y > 0.0;
      neg_im = neg_im || g.y < 0.0;
    }
  }
  if (all_zero) return HELM_ESINGULAR;
  const int last = dim - 1;
  if (glo[last].y != 0.0 || ghi[last].y != 0.0) return (pos_im && neg_im) ? HELM_EUNSUPPORTED : HELM_OK;
  if (!all_real || neg_re) return HELM_EUNSUPPORTED;
  if (c < 0.0) return HELM_OK;
  if (c == 0.0 && (glo[last].x > 0.0 || ghi[last].x > 0.0)) return HELM_OK;
  return HELM_EUNSUPPORTED;
}

int setup_impl(int dim, const int64_t* grid, const double* h, double c, long double cx, const double2* glo,
               const double2* ghi, const helm_options* opt, helm_plan** out);

}  // namespace

extern "C" {

int helm_setup(int dim, const int64_t* grid, const double* h, double omega, uint32_t abc,
               const helm_options* opt, helm_plan** out) {
  if (!out || !grid || !h || (dim != 2 && dim != 3)) return HELM_EINVAL;
  *out = nullptr;
  if (!std::isfinite(omega)) return HELM_EINVAL;
  if (abc >> (2 * dim)) return HELM_EINVAL;
  double2 glo[3], ghi[3];
  for (int j = 0; j < dim; ++j) {
    const cd gl = face_gamma(omega, (abc >> (2 * j)) & 1), gh = face_gamma(omega, (abc >> (2 * j + 1)) & 1);
    glo[j] = make_double2(gl.real(), gl.imag());
    ghi[j] = make_double2(gh.real(), gh.imag());
  }
  // c = omega^2; the shifts take it to extended precision
  return setup_impl(dim, grid, h, omega * omega, (long double)omega * (long double)omega, glo, ghi, opt, out);
}

int helm_setup_general(int dim, const int64_t* grid, const double* h, double c, const double* gamma,
                       const helm_options* opt, helm_plan** out) {
  if (!out || !grid || !h || !gamma || (dim != 2 && dim != 3)) return HELM_EINVAL;
  *out = nullptr;
  double2 glo[3], ghi[3];
  for (int j = 0; j < dim; ++j) {
    glo[j] = make_double2(gamma[4 * j], gamma[4 * j + 1]);
    ghi[j] = make_double2(gamma[4 * j + 2], gamma[4 * j + 3]);
  }
  return setup_impl(dim, grid, h, c, (long double)c, glo, ghi, opt, out);
}

}  // extern "C"

namespace {

int setup_impl(int dim, const int64_t* grid, const double* h, double c, long double cx, const double2* glo,
               const double2* ghi, const helm_options* opt, helm_plan** out) {
  for (int j = 0; j < dim; ++j)
    if (grid[j] < 3 || grid[j] > (1 << 24) || !(h[j] > 0.0) || !std::isfinite(h[j])) return HELM_EINVAL;
  const int chk = check_coefficients(dim, c, glo, ghi);
  if (chk != HELM_OK) return chk;
  const int last = dim - 1;
  std::unique_ptr<helm_plan> p(new (std::nothrow) helm_plan());
  if (!p) return HELM_ENOMEM;
  p->dim = dim;
  p->cz = c;
  p->czx = cx;
  for (int j = 0; j < dim; ++j) {
    p->glo[j] = glo[j];
    p->ghi[j] = ghi[j];
  }
  helm_default_options(&p->opt);
  if (opt) p->opt = *opt;
  if (p->opt.precision != HELM_PREC_FP64 && p->opt.precision != HELM_PREC_MIXED) return HELM_EINVAL;
  if (p->opt.max_iter < 0 || !(p->opt.tol >= 0.0)) return HELM_EINVAL;
  const int tf = p->opt.transform;
  if (tf != HELM_TRANSFORM_AUTO && tf != HELM_TRANSFORM_FFT && tf != HELM_TRANSFORM_DENSE) return HELM_EINVAL;
  const int bmode = p->opt.boundary;
  if (bmode != HELM_BOUNDARY_AUTO && bmode != HELM_BOUNDARY_LINES && bmode != HELM_BOUNDARY_TABLES)
    return HELM_EINVAL;
  const int emode = p->opt.eigen;
  if (emode != HELM_EIGEN_AUTO && emode != HELM_EIGEN_HOST && emode != HELM_EIGEN_DEVICE) return HELM_EINVAL;
  const bool want_tab = dim == 3 && bmode != HELM_BOUNDARY_LINES && tf != HELM_TRANSFORM_DENSE;
  if (p->opt.tune_cache) p->tune_path = p->opt.tune_cache;
  p->opt.tune_cache = nullptr;
  bool dense_ok = tf != HELM_TRANSFORM_FFT;
  for (int j = 0; j < dim - 1; ++j) dense_ok = dense_ok && grid[j] <= HELM_DENSE_MAX;
  if (tf == HELM_TRANSFORM_DENSE && !dense_ok) return HELM_EUNSUPPORTED;
  for (int j = 0; j < dim; ++j) {
    p->grid[j] = grid[j];
    p->h[j] = h[j];
  }
  // size limits of this build, checked before any device call: line axis
  // <= 4096 nodes (at most 512 lanes of 8 rows) or 4097 (512 lanes and the
  // extra row), periodised lengths whose transform splits into two passes of
  // <= 512 (power of two <= 2^18, or a chirp-z convolution length <= 2^18)
  if (grid[last] > 4097) return HELM_EUNSUPPORTED;
  for (int j = 0; j < dim - 1; ++j) {
    int64_t M = 1;
    while (M < (is_pow2(grid[j]) ? grid[j] : 2 * grid[j] - 1)) M <<= 1;
    if (M > 512 * 512) return HELM_EUNSUPPORTED;
  }
  if (hipGetDevice(&p->device) != hipSuccess) return HELM_EDEVICE;
  p->nper = dim - 1;
  p->nL = (int)grid[last];
  p->hL = h[last];
  p->kLo = corner_h(glo[last], h[last]);
  p->kHi = corner_h(ghi[last], h[last]);
  if (p->nL > 4097) return HELM_EUNSUPPORTED;
  for (int j = 0; j < p->nper; ++j) {
    PAxis& a = p->ax[j];
    a.n = (int)grid[j];
    a.h = h[j];
    a.glo = glo[j];
    a.ghi = ghi[j];
    if (is_pow2(a.n)) {
      pow2_split(a.n, &a.na, &a.nbp);
      if (a.na > 512 || a.nbp > 512) return HELM_EUNSUPPORTED;
    } else {
      const int bst = setup_bluestein(a);
      if (bst != HELM_OK) return bst;
    }
    std::vector<cd> vfull, lamlo;
    // whole eigenvectors: both axes for the dense transform, the inner one
    // for the boundary tables
    const bool vecs = dense_ok || (want_tab && j == 1);
    if (emode == HELM_EIGEN_HOST) {
      const int st = eig1d(a.n, a.h, cd(a.glo.x, a.glo.y), cd(a.ghi.x, a.ghi.y), a.lamA, a.va0, a.va1,
                           vecs ? &vfull : nullptr, &lamlo);
      if (st != HELM_OK) return st;
      if (vecs) {
        const int ast = upload_eigvecs(a, vfull);
        if (ast != HELM_OK) return ast;
      }
    } else {
      EigVecOut vo{};
      if (vecs) {
        const int ast = eigvec_buffers(a, &vo);
        if (ast != HELM_OK) return ast;
      }
      const int st = eig1d_device(a.n, a.h, cd(a.glo.x, a.glo.y), cd(a.ghi.x, a.ghi.y), a.lamA, a.va0, a.va1, lamlo,
                                  vecs ? &vo : nullptr, nullptr);
      if (st != HELM_OK) return st;
    }
    a.lamAx.resize(a.n);
    for (int l = 0; l < a.n; ++l)
      a.lamAx[l] = std::complex<long double>((long double)a.lamA[l].real() + lamlo[l].real(),
                                             (long double)a.lamA[l].imag() + lamlo[l].imag());
    std::vector<double2> buf;
    std::vector<double> invmu;
    fill_axis_tables_host(a, cx, buf, invmu);
    const size_t nb2 = (size_t)a.n * 8 * sizeof(double2);
    if (a.tab.ensure(nb2 + (size_t)a.n * sizeof(double)) != hipSuccess) return HELM_ENOMEM;
    if (upload(a.tab.p, buf.data(), nb2) != hipSuccess) return HELM_EDEVICE;
    if (upload((char*)a.tab.p + nb2, invmu.data(), (size_t)a.n * sizeof(double)) != hipSuccess)
      return HELM_EDEVICE;
    double2* t = a.tab.as<double2>();
    a.sigB = t;
    a.sigA = t + a.n;
    a.genB0 = t + 2 * a.n;
    a.genB1 = t + 3 * a.n;
    a.redB0 = t + 4 * a.n;
    a.redB1 = t + 5 * a.n;
    a.va0d = t + 6 * a.n;
    a.va1d = t + 7 * a.n;
    a.invmu = reinterpret_cast<double*>((char*)a.tab.p + nb2);
  }
  // Line-matrix families (outer branch, inner branch): the shift
  // sigma = lambda_outer + lambda_inner - w^2 of every line, formed in extended
  // precision and rounded once (near-resonant modes would otherwise lose
  // digits to cancellation against w^2), and the LU factors (reciprocal Thomas
  // pivots; Section 4.1.2 computes the LU decompositions of H_B and H_A at
  // initialisation).
  {
    const int nO = dim == 2 ? 1 : p->ax[0].n;
    const int nI = p->ax[dim - 2].n;
    const int fam = dim == 2 ? 2 : 4;
    const PAxis& inner = p->ax[dim - 2];
    const size_t pairs = (size_t)nO * nI;
    std::vector<double2> hs(pairs * fam);
    const long double w2x = p->czx;
    for (int k = 0; k < fam; ++k) {
      for (int l = 0; l < nO; ++l) {
        std::complex<long double> so(0.0L, 0.0L);
        if (dim == 3) so = (k & 2) ? p->ax[0].lamAx[l] : std::complex<long double>(p->ax[0].lamBx[l], 0.0L);
        for (int m = 0; m < nI; ++m) {
          const std::complex<long double> si =
              (k & 1) ? inner.lamAx[m] : std::complex<long double>(inner.lamBx[m], 0.0L);
          const std::complex<long double> sg = so + si - w2x;
          hs[pairs * k + (size_t)l * nI + m] = make_double2((double)sg.real(), (double)sg.imag());
        }
      }
    }
    if (p->sigtab.ensure(hs.size() * sizeof(double2)) != hipSuccess) return HELM_ENOMEM;
    if (upload(p->sigtab.p, hs.data(), hs.size() * sizeof(double2)) != hipSuccess) return HELM_EDEVICE;
    int P, c, NT;
    lines_geometry(p->nL, &P, &c, &NT);
    const size_t per = pairs * P;
    if (p->factors.ensure(per * fam * sizeof(double2)) != hipSuccess) return HELM_ENOMEM;
    for (int k = 0; k < fam; ++k) {
      p->sig[k] = p->sigtab.as<double2>() + pairs * k;
      LineArgs la;
      la.nb = 1;
      la.nO = nO;
      la.nI = nI;
      la.nL = p->nL;
      la.sTab = p->sig[k];
      la.hL = p->hL;
      la.kLo = p->kLo;
      la.kHi = p->kHi;
      double2* dst = p->factors.as<double2>() + per * k;
      if (launch_line_factors(la, dst, nullptr) != hipSuccess) return HELM_EDEVICE;
      p->seed[k] = dst;
    }
    if (hipDeviceSynchronize() != hipSuccess) return HELM_EDEVICE;
  }
  if (dim == 3 && tf != HELM_TRANSFORM_DENSE) {
    const int lrc = tune_layout(p.get());
    if (lrc != HELM_OK) return lrc;
  }
  if (want_tab) {
    const int brc = setup_boundary_tables(p.get());
    if (brc != HELM_OK) return brc;
  }
  if (tf != HELM_TRANSFORM_DENSE) {
    const int frc = tune_fft_tile(p.get());
    if (frc != HELM_OK) return frc;
    const int crc = tune_chirp(p.get());
    if (crc != HELM_OK) return crc;
  }
  if (prepare_roots(p.get()) != HELM_OK) return HELM_ENOMEM;
  if (hipHostMalloc(reinterpret_cast<void**>(&p->h_norms_pin), 2 * HELM_STATIC_MAX_RHS * sizeof(double),
                    hipHostMallocDefault) != hipSuccess) {
    p->h_norms_pin = nullptr;
    return HELM_ENOMEM;
  }
  {
    const int src = static_workspace(p->device, &p->static_ws);
    if (src != HELM_OK) return src;
  }
  if (tf == HELM_TRANSFORM_DENSE) {
    p->dense = 1;
  } else if (tf == HELM_TRANSFORM_AUTO && dense_ok) {
    const int trc = autotune_transform(p.get());
    if (trc != HELM_OK) return trc;
  }
  p->rep.status = HELM_OK;
  p->rep.rel_residual_max = -1;
  p->rep.rel_residual_first = -1;
  *out = p.release();
  return HELM_OK;
}

}  // namespace

extern "C" {

int helm_solve(helm_plan* p, const void* f, void* u, int nrhs, void* stream) {
  return helm::solve_entry(p, f, u, nrhs, reinterpret_cast<hipStream_t>(stream), true);
}

int helm_solve_static(helm_plan* p, const void* f, void* u, int nrhs, void* stream) {
  return helm::solve_static(p, f, u, nrhs, reinterpret_cast<hipStream_t>(stream));
}

int helm_report_get(const helm_plan* p, helm_report* out) {
  if (!p || !out) return HELM_EINVAL;
  *out = p->rep;
  return HELM_OK;
}

int helm_residual(helm_plan* p, const void* u, const void* f, void* r, double* rel_res, int nrhs,
                  void* stream) {
  if (!p || !u || !f || !rel_res || nrhs < 1) return HELM_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t N = npoints(p);
  const auto before = workspace_addrs(p);
  const bool ok = p->scratch.ensure((size_t)residual_scratch_len(p->dim, p->grid, nrhs) * sizeof(double)) ==
                      hipSuccess &&
                  p->norms.ensure((size_t)nrhs * 2 * sizeof(double)) == hipSuccess;
  if (workspace_addrs(p) != before) ++p->ws_gen;
  if (!ok) return HELM_ENOMEM;
  p->h_norms.resize(2 * nrhs);
  (void)N;
  double mx = 0;
  std::vector<double> rel;
  const int rc = residual_norms(p, reinterpret_cast<const double2*>(u), reinterpret_cast<const double2*>(f), r,
                                ST_C128, nrhs, st, &mx, &rel);
  for (int b = 0; b < nrhs; ++b) rel_res[b] = rc == HELM_OK ? rel[b] : NAN;
  return rc;
}

int helm_profile(helm_plan* p, int on) {
  if (!p) return HELM_EINVAL;
  p->prof = on != 0;
  return HELM_OK;
}

int helm_kernel_stats_get(helm_plan* p, helm_kernel_stats* out, int reset) {
  if (!p || !out) return HELM_EINVAL;
  const hipError_t e = collect_events(p);
  if (e != hipSuccess) return map_err(e);
  *out = p->kst;
  if (reset) p->kst = helm_kernel_stats{};
  return HELM_OK;
}

const char* helm_kernel_name(int k) {
  static const char* names[HELM_NKERNELS] = {
      "fft_pass_kernel<double2>", "fft_pass_kernel<float2>", "lines_kernel",    "inner_mid_kernel",
      "sum_to_planes_kernel",     "outer_mid_kernel",        "residual_kernel", "dense_kernel",
      "cap_apply_kernel"};
  return (k >= 0 && k < HELM_NKERNELS) ? names[k] : nullptr;
}

void helm_destroy(helm_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  delete p;
}

int helm_batch_create(helm_plan* const* plans, int count, int max_nrhs, helm_batch** out) {
  if (!out) return HELM_EINVAL;
  *out = nullptr;
  if (!plans || count < 1 || max_nrhs < 1) return HELM_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HELM_EDEVICE;
  std::vector<helm_plan*> v(plans, plans + count);
  for (int i = 0; i < count; ++i) {
    if (!v[i] || v[i]->device != dev) return HELM_EINVAL;
    for (int j = 0; j < i; ++j)
      if (v[j] == v[i]) return HELM_EINVAL;  // a plan's workspace serves one problem
  }
  std::unique_ptr<helm_batch> b(new (std::nothrow) helm_batch());
  if (!b) return HELM_ENOMEM;
  b->plans = v;
  b->max_nrhs = max_nrhs;
  b->device = dev;
  for (helm_plan* p : v) {
    const bool mixed = p->opt.precision == HELM_PREC_MIXED;
    const int rc = ensure_workspace(p, max_nrhs, mixed, mixed || p->opt.check);
    if (rc) return rc;
  }
  const int ns = std::min(count, kBatchMaxBranches);
  for (int k = 0; k < ns; ++k) {
    hipStream_t s;
    hipEvent_t e;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HELM_EDEVICE;
    b->side.push_back(s);
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return HELM_EDEVICE;
    b->join.push_back(e);
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) return HELM_EDEVICE;
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return HELM_EDEVICE;
  *out = b.release();
  return HELM_OK;
}

int helm_batch_solve(helm_batch* b, const void* const* f, void* const* u, const int* nrhs, void* stream) {
  if (!b || !f || !u || !nrhs) return HELM_EINVAL;
  const int n = (int)b->plans.size();
  for (int i = 0; i < n; ++i) {
    if (!f[i] || !u[i] || f[i] == u[i] || nrhs[i] < 1 || nrhs[i] > b->max_nrhs) return HELM_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  bool same = b->exec && b->kst == st;
  for (int i = 0; same && i < n; ++i)
    same = b->kf[i] == f[i] && b->ku[i] == u[i] && b->kn[i] == nrhs[i] && b->kgen[i] == b->plans[i]->ws_gen;
  if (!same) {
    b->drop_graph();
    // Eager solves first: they create every lazily built table (twiddles,
    // chirps) outside the capture and give the refinement depth to capture:
    // one step more than these inputs needed, at least 2, at most max_iter.
    b->steps.assign(n, 0);
    for (int i = 0; i < n; ++i) {
      helm_plan* p = b->plans[i];
      const int rc = helm::solve_entry(p, f[i], u[i], nrhs[i], st, false);
      if (rc != HELM_OK && rc != HELM_ENOCONV) return rc;
      b->steps[i] = std::min(p->opt.max_iter, std::max(2, p->rep.iterations + 1));
    }
    if (hipStreamSynchronize(st) != hipSuccess) return HELM_EDEVICE;
    // longest problems first, each onto the branch with the least work
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto work = [&](int i) { return (double)npoints(b->plans[i]) * nrhs[i] * (1 + b->steps[i]); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    // one graph with `ns` parallel branches (side streams)
    auto capture = [&](int ns, hipGraph_t* out_g) -> int {
      std::vector<double> load(ns, 0.0);
      int rc = HELM_OK;
      hipStream_t cs = b->cap;
      if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) return HELM_EDEVICE;
      do {
        if (hipEventRecord(b->fork, cs) != hipSuccess) { rc = HELM_EDEVICE; break; }
        for (int k = 0; k < ns; ++k)
          if (hipStreamWaitEvent(b->side[k], b->fork, 0) != hipSuccess) rc = HELM_EDEVICE;
        if (rc) break;
        for (int i : order) {
          const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
          load[k] += work(i);
          rc = enqueue_device_ir(b->plans[i], reinterpret_cast<const double2*>(f[i]),
                                 reinterpret_cast<double2*>(u[i]), nrhs[i], b->steps[i], b->steps[i], nullptr,
                                 b->side[k]);
          if (rc) break;
        }
        // join every side stream back (also after an error, so that the
        // capture can end)
        for (int k = 0; k < ns; ++k) {
          if (hipEventRecord(b->join[k], b->side[k]) != hipSuccess) rc = HELM_EDEVICE;
          if (hipStreamWaitEvent(cs, b->join[k], 0) != hipSuccess) rc = HELM_EDEVICE;
        }
      } while (false);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(cs, &g);
      if (rc || ce != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc ? rc : HELM_EDEVICE;
      }
      *out_g = g;
      return HELM_OK;
    };
    // The number of branches is tuned: the candidates (all side streams, a
    // half, a quarter) are captured and timed once each on these inputs (a
    // launch is a whole solve, so the timing runs also leave u solved), the
    // fastest is kept, and the choice is appended to the first plan's tune
    // cache under the batch's shape signature and read back from there.
    const int nmax = (int)b->side.size();
    const std::string bkey = batch_key(b, nrhs);
    const std::string& tpath = b->plans[0]->tune_path;
    std::vector<int> cands;
    int cached = 0;
    if (b->branches > 0) {
      cands.push_back(b->branches);
    } else if (!tpath.empty() && tune_lookup(tpath, bkey, "branches=", &cached) && cached >= 1 && cached <= nmax) {
      cands.push_back(cached);
    } else {
      for (int c = nmax; c >= 1 && (int)cands.size() < 3; c /= 2) cands.push_back(c);
    }
    std::vector<float> times;
    int best = -1;
    float best_ms = 0;
    for (int c : cands) {
      hipGraph_t g = nullptr;
      int rc = capture(c, &g);
      if (rc) return rc;
      hipGraphExec_t ex = nullptr;
      if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return HELM_EDEVICE;
      }
      float ms = 0;
      if (cands.size() > 1) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) rc = HELM_EDEVICE;
        if (!rc && hipEventCreate(&e1) != hipSuccess) {
          (void)hipEventDestroy(e0);
          rc = HELM_EDEVICE;
        }
        if (!rc) {
          if (hipEventRecord(e0, st) != hipSuccess || hipGraphLaunch(ex, st) != hipSuccess ||
              hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = HELM_EDEVICE;
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
        }
      }
      times.push_back(ms);
      if (!rc && (best < 0 || ms < best_ms)) {
        b->drop_graph();
        b->graph = g;
        b->exec = ex;
        best = c;
        best_ms = ms;
      } else {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
      }
      if (rc) {
        b->drop_graph();
        return rc;
      }
    }
    if (cands.size() > 1 && !tpath.empty()) {
      FILE* tf = std::fopen(tpath.c_str(), "a");
      if (tf) {
        std::fprintf(tf, "helm-tune %s branches=%d", bkey.c_str(), best);
        for (size_t k = 0; k < cands.size(); ++k) std::fprintf(tf, " b%d_ms=%.6g", cands[k], times[k]);
        std::fprintf(tf, "\n");
        std::fclose(tf);
      }
    }
    b->branches = best;
    b->kf.assign(f, f + n);
    b->ku.assign(u, u + n);
    b->kn.assign(nrhs, nrhs + n);
    b->kgen.resize(n);
    for (int i = 0; i < n; ++i) b->kgen[i] = b->plans[i]->ws_gen;
    b->kst = st;
  }
  if (hipGraphLaunch(b->exec, st) != hipSuccess) return HELM_EDEVICE;
  b->last = st;
  return HELM_OK;
}

int helm_batch_report_get(helm_batch* b, int i, helm_report* out) {
  if (!b || !out || i < 0 || i >= (int)b->plans.size()) return HELM_EINVAL;
  if (!b->exec) return HELM_EINVAL;
  if (hipStreamSynchronize(b->last) != hipSuccess) return HELM_EDEVICE;
  helm_plan* p = b->plans[i];
  IrCtl c;
  if (hipMemcpy(&c, p->ctl.p, sizeof(IrCtl), hipMemcpyDeviceToHost) != hipSuccess) return HELM_EDEVICE;
  helm_report r{};
  r.status = c.status;
  r.iterations = c.iters;
  r.precision = p->opt.precision;
  r.transform = p->dense ? HELM_TRANSFORM_DENSE : HELM_TRANSFORM_FFT;
  r.boundary = boundary_used(p, b->kn[i]);
  r.nrhs = b->kn[i];
  r.rel_residual_max = c.rel_last;
  r.rel_residual_first = c.rel_first;
  *out = r;
  return HELM_OK;
}

void helm_batch_destroy(helm_batch* b) { delete b; }

}  // extern "C"
