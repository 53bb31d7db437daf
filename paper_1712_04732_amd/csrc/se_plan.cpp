// Host planner and C ABI of the Spectral Ewald k-space library (se.h).
//
// The planner applies the paper's parameter rules (Section 3.3, Section 6),
// builds every FP64 table once (PKB coefficients of Section 4.1, separable
// scaling vectors and Green's-function tables of Eq. scale / Section 3.1),
// runs Algorithm 3 on the GPU for free space, lays out the evaluation's work
// buffers in a caller-owned workspace and records the launch sequence of
// Algorithm 4 for one system.  se_eval only enqueues kernels.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/se.h"
#include "se_internal.h"

// Stand-in base of a plan's work pointers before a workspace is bound (the
// first page, which no device allocation occupies).
constexpr uintptr_t kWsStandIn = 4096;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

int smooth_even_up(long n) {
  long m = std::max(2L, n);
  if (m % 2) ++m;
  for (;; m += 2) {
    long r = m;
    for (int p : {2, 3, 5, 7})
      while (r % p == 0) r /= p;
    if (r == 1) return (int)m;
  }
}

bool is_smooth(long n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}

// Radix sequence for the Stockham stages: the fewest stages over the radices
// 2-9 (each stage is one LDS round trip and one barrier; radices 6 and 9 are
// composite butterflies, 2 x 3 and 3 x 3, in registers), found by a search
// over the divisors of n.  Where the prime radices 8, 4, 2, 3, 5, 7 taken
// greedily in that order need no more stages, that sequence; otherwise,
// among the shortest, the one with the most eights, then nines, sixes,
// sevens, fives and fours, run in the order 8, 4, 2, 9, 6, 3, 5, 7.
bool radix_plan(int n, int* rad, int* nst) {
  if (n < 1 || !is_smooth(n)) return false;
  int greedy[64], ng = 0;
  int rem = n;
  for (int r : {8, 4, 2, 3, 5, 7})
    for (; rem % r == 0 && ng < 64; rem /= r) greedy[ng++] = r;
  static const int pref[] = {8, 9, 6, 7, 5, 4, 3, 2};
  std::vector<int> best(n + 1, -1);   // fewest stages for each divisor m of n
  best[1] = 0;
  for (int m = 2; m <= n; ++m) {
    if (n % m) continue;
    for (int r : pref)
      if (m % r == 0 && best[m / r] >= 0 && (best[m] < 0 || best[m / r] + 1 < best[m])) best[m] = best[m / r] + 1;
  }
  if (best[n] < 0 || best[n] > se::kMaxStages) return false;
  if (ng == best[n]) {
    for (int k = 0; k < ng; ++k) rad[k] = greedy[k];
    *nst = ng;
    return true;
  }
  int cnt[10] = {0};
  for (int m = n; m > 1;) {
    for (int r : pref)
      if (m % r == 0 && best[m / r] == best[m] - 1) {
        ++cnt[r];
        m /= r;
        break;
      }
  }
  int k = 0;
  for (int r : {8, 4, 2, 9, 6, 3, 5, 7})
    for (int i = 0; i < cnt[r]; ++i) rad[k++] = r;
  *nst = k;
  return true;
}

// Modified Bessel function I0 by its power series sum (x^2/4)^k / (k!)^2.
double bessel_i0(double x) {
  const double y = 0.25 * x * x;
  double term = 1.0, s = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= y / ((double)k * k);
    s += term;
    if (term < 1e-17 * s) break;
  }
  return s;
}

// Modified Bessel function I1 by its power series (x/2) sum (x^2/4)^k / (k! (k+1)!).
double bessel_i1(double x) {
  const double y = 0.25 * x * x;
  double term = 0.5 * x, s = term;
  for (int k = 1; k < 500; ++k) {
    term *= y / ((double)k * (k + 1));
    s += term;
    if (std::fabs(term) < 1e-17 * std::fabs(s)) break;
  }
  return s;
}

// KB window in grid units u (w = P/2), Eq. (kaiser_window).
double kb_window(double u, int P, double beta) {
  const double z = 2.0 * u / P;
  if (std::fabs(z) > 1.0) return 0.0;
  return bessel_i0(beta * std::sqrt(1.0 - z * z)) / bessel_i0(beta);
}

// d/du of the KB window (grid units): -I1(beta s) beta z (2/P) / (s I0(beta)),
// s = sqrt(1 - z^2); 0 outside the support.
double kb_window_du(double u, int P, double beta) {
  const double z = 2.0 * u / P;
  if (std::fabs(z) >= 1.0) return 0.0;
  const double s = std::sqrt(1.0 - z * z);
  return -bessel_i1(beta * s) * beta * z * (2.0 / P) / (s * bessel_i0(beta));
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double t = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = -t;
    x[n - 1 - i] = t;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// Fourier transform of the ES window, Eq. (expsemicirc_window), which has no
// closed form (Section 4): with x = w sin(theta),
//   int_{-w}^{w} e^{beta (sqrt(1 - (x/w)^2) - 1)} cos(k x) dx
//     = w int_{-pi/2}^{pi/2} e^{beta (cos theta - 1)} cos(k w sin theta) cos theta dtheta,
// a smooth integrand, by 256-point Gauss-Legendre quadrature.
double es_ft(double k, double w, double beta) {
  static std::vector<double> gx, gw;
  static std::once_flag once;
  std::call_once(once, [] { gauss_legendre(256, gx, gw); });
  double s = 0.0;
  for (size_t i = 0; i < gx.size(); ++i) {
    const double th = 0.5 * kPi * gx[i];
    s += gw[i] * std::exp(beta * (std::cos(th) - 1.0)) * std::cos(k * w * std::sin(th)) * std::cos(th);
  }
  return 0.5 * kPi * w * s;
}

// 1D Fourier transform of the window used in the scaling step: Eq. (kaiser_ft)
// for KB, the untruncated Gaussian transform for the Gaussian (Section 4).
double window_ft(double k, double h, int P, int window, double shape) {
  const double w = P * h / 2.0;
  if (window == SE_WIN_GAUSSIAN) return std::sqrt(kPi / shape) * w * std::exp(-k * k * w * w / (4.0 * shape));
  if (window == SE_WIN_ES) return es_ft(k, w, shape);
  const double d = shape * shape - k * k * w * w;
  const double sd = std::sqrt(std::fabs(d));
  double r;
  if (sd == 0.0)
    r = 1.0;
  else
    r = d > 0 ? std::sinh(sd) / sd : std::sin(sd) / sd;
  return 2.0 * w * r / bessel_i0(shape);
}

// Solve V c = b for the (m x m) system by Gaussian elimination with partial pivoting.
bool solve(std::vector<double> A, std::vector<double> b, int m, std::vector<double>& x) {
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(A[r * m + c]) > std::fabs(A[piv * m + c])) piv = r;
    if (A[piv * m + c] == 0.0) return false;
    if (piv != c) {
      for (int j = 0; j < m; ++j) std::swap(A[c * m + j], A[piv * m + j]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < m; ++r) {
      const double f = A[r * m + c] / A[c * m + c];
      for (int j = c; j < m; ++j) A[r * m + j] -= f * A[c * m + j];
      b[r] -= f * b[c];
    }
  }
  x.assign(m, 0.0);
  for (int r = m - 1; r >= 0; --r) {
    double s = b[r];
    for (int j = r + 1; j < m; ++j) s -= A[r * m + j] * x[j];
    x[r] = s / A[r * m + r];
  }
  return true;
}

// PKB coefficients (Section 4.1): on subinterval i of [-w, w] the KB window
// is interpolated at the nu+1 Chebyshev points xbar_k = cos(pi (k - 1/2)/(nu+1))
// by sum_j c_ij xbar^j (Eqs. polynomial-ansatz, polynomial-linsys).
bool pkb_coefficients(int P, double beta, int nu, std::vector<double>& c,
                      double (*fn)(double, int, double) = kb_window) {
  const int m = nu + 1;
  std::vector<double> V(m * m), xb(m);
  for (int k = 0; k < m; ++k) {
    xb[k] = std::cos(kPi * (k + 0.5) / m);
    double p = 1.0;
    for (int j = 0; j < m; ++j) {
      V[k * m + j] = p;
      p *= xb[k];
    }
  }
  c.assign((size_t)P * m, 0.0);
  for (int i = 0; i < P; ++i) {
    std::vector<double> rhs(m), sol;
    for (int k = 0; k < m; ++k) rhs[k] = fn(-P / 2.0 + i + (xb[k] + 1.0) / 2.0, P, beta);
    if (!solve(V, rhs, m, sol)) return false;
    for (int j = 0; j < m; ++j) c[(size_t)i * m + j] = sol[j];
  }
  return true;
}

// Modified Green's functions at vanishing periodic wavenumber (Section 3.1).
double g2p_zero(double kap, double R) {  // Eq. (G_hat_2d)
  kap = std::fabs(kap);
  if (kap == 0.0) return -R * R / 2.0;
  return (1.0 - std::cos(R * kap) - R * kap * std::sin(R * kap)) / (kap * kap);
}
double g1p_zero(double kap, double R) {  // Eq. (G_hat_1d)
  if (kap == 0.0) return R * R / 4.0 * (1.0 - 2.0 * std::log(R));
  return (1.0 - ::j0(R * kap)) / (kap * kap) - R * std::log(R) * ::j1(R * kap) / kap;
}

int signed_freq(int t, int n) { return t < (n + 1) / 2 ? t : t - n; }

const char* kStatusText[] = {"ok",
                             "invalid argument",
                             "invalid parameters",
                             "charges are not neutral",
                             "a free-direction coordinate lies outside [0, L)",
                             "non-finite position or charge",
                             "HIP runtime error",
                             "device allocation failed",
                             "not supported",
                             "no workspace bound, or the workspace is too small or misaligned"};

}  // namespace

struct se_plan {
  se_params p{};
  se_plan_info info{};
  bool f64 = true;
  long n_max = 0;
  int device = 0;
  se::GridGeom geom{};
  se::EvalBuffers buf{};
  std::vector<void*> allocs;
  std::vector<se::FftPass> passes;
  // force method 2: for each direction d, the fused pass with i k_d and the
  // two inverse passes, writing shadow copies of the spectrum buffers
  std::vector<se::FftPass> ik_passes;
  std::vector<std::pair<char*, size_t>> spec;   // spectrum buffers (workspace)
  int ntiles = 0;
  int nsbtot = 0;
  // tracing: HIP event pairs around launches of SE_PROFILE evaluations
  struct ProfRec {
    int site;
    int ev;
    double bytes, flops;
  };
  std::vector<hipEvent_t> evpool;
  int ev_used = 0;
  std::vector<ProfRec> prof;
  size_t lds_limit = 65536;   // soft budget: keeps several workgroups per CU
  int fft_cap = 0;            // samples per FFT workgroup (0: by precision)
  size_t lds_max = 65536;     // device maximum per workgroup
  size_t bytes = 0;           // device memory the plan owns (tables)
  // Workspace: every buffer of an evaluation (particles, grid, spectra,
  // partial sums) lies in one caller-owned block.  During planning the
  // buffers are laid out as offsets from a stand-in base (kWsStandIn, never a
  // device address); binding a block moves every work pointer to it.
  size_t ws_bytes = 0;
  uintptr_t ws_base = kWsStandIn;
  bool ws_bound = false;

  ~se_plan() {
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    for (void* a : allocs) (void)hipFree(a);
  }

  // A work buffer of n bytes at the next 256-byte boundary of the workspace.
  void* walloc(size_t n) {
    const size_t o = (ws_bytes + 255) & ~(size_t)255;
    ws_bytes = o + std::max<size_t>(n, 16);
    return (void*)(ws_base + o);
  }

  // Move every work pointer from the current base to 'base'.
  void rebase(uintptr_t base) {
    const uintptr_t lo = ws_base, hi = ws_base + ws_bytes;
    auto mv = [&](auto& ptr) {
      const uintptr_t v = (uintptr_t)ptr;
      if (v >= lo && v < hi) ptr = (std::remove_reference_t<decltype(ptr)>)(v - lo + base);
    };
    se::EvalBuffers& b = buf;
    mv(b.sb_count); mv(b.sb_start); mv(b.sb_cursor); mv(b.p_key); mv(b.p_cell); mv(b.p_frac);
    mv(b.s_cell); mv(b.s_idx); mv(b.s_fq); mv(b.bsum); mv(b.stage); mv(b.qpart); mv(b.epart);
    mv(b.red); mv(b.grid); mv(b.vjp_phi); mv(b.vjp_grad);
    for (auto* list : {&passes, &ik_passes})
      for (se::FftPass& ps : *list)
        for (se::FftClass& c : ps.cls) {
          mv(c.in);
          mv(c.out);
        }
    for (auto& sb : spec) mv(sb.first);
    ws_base = base;
  }

  void* dalloc(size_t n) {
    void* ptr = nullptr;
    if (n == 0) n = 16;
    if (hipMalloc(&ptr, n) != hipSuccess) return nullptr;
    allocs.push_back(ptr);
    bytes += n;
    return ptr;
  }

  // Upload an FP64 host table in the compute precision.
  const void* upload(const std::vector<double>& v) {
    const size_t esz = f64 ? 8 : 4;
    void* d = dalloc(v.size() * esz);
    if (!d) return nullptr;
    hipError_t e;
    if (f64) {
      e = hipMemcpy(d, v.data(), v.size() * 8, hipMemcpyHostToDevice);
    } else {
      std::vector<float> f(v.begin(), v.end());
      e = hipMemcpy(d, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    }
    return e == hipSuccess ? d : nullptr;
  }

  // Twiddles exp(-2 pi i k/n), k = 0..n-1, interleaved complex, evaluated in
  // extended precision and rounded once to the compute precision; one table
  // per (length, precision), shared by the passes of the plan.
  std::vector<std::pair<long, const void*>> twc;
  const void* twiddles(int n) {
    const long key = 2L * n + (f64 ? 1 : 0);
    for (const auto& e : twc)
      if (e.first == key) return e.second;
    std::vector<double> w(2 * (size_t)n);
    const long double two_pi = 6.283185307179586476925286766559L;
    for (int k = 0; k < n; ++k) {
      const long double a = two_pi * (long double)k / (long double)n;
      w[2 * k] = (double)cosl(a);
      w[2 * k + 1] = (double)-sinl(a);
    }
    const void* d = upload(w);
    if (d) twc.emplace_back(key, d);
    return d;
  }

  // Scaling vector of a direction transformed at length n over spacing h:
  //   e^{-k^2/4xi^2} / What(k)^2 / n   with k = 2 pi m/(n h), m the signed frequency.
  // The 1/n is the inverse transform's normalisation.
  const void* sep_table(int n) {
    std::vector<double> s(n);
    for (int t = 0; t < n; ++t) {
      const double k = 2.0 * kPi * signed_freq(t, n) / (n * info.h);
      const double W = window_ft(k, info.h, p.P, p.window, p.shape);
      s[t] = std::exp(-k * k / (4.0 * p.xi * p.xi)) / (W * W) / n;
    }
    return upload(s);
  }

  // Signed wavenumbers k = 2 pi m/(n h) of a length-n transform, m the signed
  // frequency, with 0 at the Nyquist index of an even n (the derivative of a
  // real grid stays real): the factor i k of force method 2.
  const void* d_table(int n) {
    std::vector<double> s(n);
    for (int t = 0; t < n; ++t)
      s[t] = (n % 2 == 0 && t == n / 2) ? 0.0 : 2.0 * kPi * signed_freq(t, n) / (n * info.h);
    return upload(s);
  }

  const void* k2_table(int n) {
    std::vector<double> s(n);
    for (int t = 0; t < n; ++t) {
      const double k = 2.0 * kPi * signed_freq(t, n) / (n * info.h);
      s[t] = k * k;
    }
    return upload(s);
  }
};

namespace {

se::FftClass make_class(int n, int n_in, int n_out, const void* in, void* out,
                        long long in_st, long long in_s0, long long in_s1, long long out_st,
                        long long out_s0, long long out_s1) {
  se::FftClass c{};
  c.n = n;
  c.n_in = n_in;
  c.n_out = n_out;
  radix_plan(n, c.rad, &c.nst);
  c.radpack = 0;
  for (int k = 0; k < c.nst; ++k) c.radpack |= (unsigned long long)c.rad[k] << (4 * k);
  c.in = in;
  c.out = out;
  c.in_st = in_st;
  c.in_s0 = in_s0;
  c.in_s1 = in_s1;
  c.out_st = out_st;
  c.out_s0 = out_s0;
  c.out_s1 = out_s1;
  return c;
}

void add_items(std::vector<int4>& items, int cls, int b0_lo, int b0_hi, int b1_lo, int b1_hi, int B) {
  for (int b1 = b1_lo; b1 < b1_hi; ++b1)
    for (int b0 = b0_lo; b0 < b0_hi; b0 += B) items.push_back(make_int4(cls, b0, b1, std::min(B, b0_hi - b0)));
}

}  // namespace

// Work-item mapping mode of a knob value: < 0 plain order, 0 the default
// (one item range per XCD), 1 one range per XCD, c >= 2 chunks of c.
static int xcd_mode(int knob) { return knob < 0 ? 0 : (knob == 0 ? 1 : knob); }

// Finish a pass: pencils per block from the LDS budget, upload the work list.
static bool finish_pass(se_plan* pl, se::FftPass& ps, int kind, int ncls,
                        const std::vector<std::vector<int>>& ranges) {
  ps.kind = kind;
  ps.nmax = 0;
  for (int c = 0; c < ncls; ++c) ps.nmax = std::max(ps.nmax, ps.cls[c].n);
  // pencils per block B, with F complex transforms: B, or B / 2 for the
  // real passes, which pair two real pencils into one complex transform.  F
  // <= 64 is bounded by the samples cap (n F), the LDS budget (twiddles n,
  // samples n (F + 1)) and the registers of an in-place stage; among the F
  // up to that bound, the smallest that gives the fewest work items (so the
  // items of a pencil range come out even)
  const size_t esz = pl->f64 ? 16 : 8;
  const bool real = kind == se::K_R2C || kind == se::K_C2R;
  const long cap = pl->fft_cap > 0 ? pl->fft_cap : (pl->f64 ? 1024 : 2048);
  // in place unless the samples cap (or a single pencil) exceeds kFftInplaceCap
  ps.inplace = (cap <= se::kFftInplaceCap && ps.nmax <= se::kFftInplaceCap) ? 1 : 0;
  auto lds_of = [&](long F) { return esz * (size_t)ps.nmax * (1 + (ps.inplace ? 1 : 2) * (F + 1)); };
  // in place, every stage of every class keeps its butterflies within the
  // registers the kernel holds for them (kFftIpIters)
  auto fits_regs = [&](long F) {
    if (!ps.inplace) return true;
    for (int c = 0; c < ncls; ++c)
      for (int k = 0; k < ps.cls[c].nst; ++k) {
        const int R = ps.cls[c].rad[k];
        if ((long)(ps.cls[c].n / R) * F > (long)se::kFftIpIters(R) * se::kFftBlock) return false;
      }
    return true;
  };
  if (!fits_regs(1)) ps.inplace = 0;   // a single pencil needs more: alternate two buffers
  int fmax = 1;
  while (fmax < 64) {
    const long F = fmax + 1;
    if ((long)ps.nmax * F > cap || lds_of(F) > std::min(pl->lds_limit, se::kFftLdsSoft) || !fits_regs(F)) break;
    ++fmax;
  }
  if (lds_of(fmax) > pl->lds_max) return false;
  auto items_of = [&](long B) {
    long k = 0;
    for (const auto& r : ranges) k += (long)(r[4] - r[3]) * ((r[2] - r[1] + B - 1) / B);
    return k;
  };
  int fb = fmax;
  long best = items_of(real ? 2L * fmax : fmax);
  for (int F = fmax - 1; F >= 1; --F) {
    const long k = items_of(real ? 2L * F : F);
    if (k <= best) {
      best = k;
      fb = F;
    }
  }
  ps.B = real ? 2 * fb : fb;
  // twiddle tables; 64-bit offsets if the B pencils of a workgroup span 4 GiB
  ps.wide = 0;
  for (int c = 0; c < ncls; ++c) {
    se::FftClass& k = ps.cls[c];
    k.tw = pl->twiddles(k.n);
    if (!k.tw) return false;
    const long double span_in = ((long double)ps.B * k.in_s0 + (long double)k.n * k.in_st) * esz;
    const long double span_out = ((long double)ps.B * k.out_s0 + (long double)k.n * k.out_st) * esz;
    if (std::max(span_in, span_out) >= 4294967296.0L) ps.wide = 1;
  }
  ps.xcd = xcd_mode(pl->p.xcd_fft);
  std::vector<int4> items;
  for (const auto& r : ranges) add_items(items, r[0], r[1], r[2], r[3], r[4], ps.B);
  ps.nitems = (int)items.size();
  // algorithmic counts: every input sample read once, every output sample
  // written once; 5 n log2 n flops per complex length-n transform
  {
    const double re = pl->f64 ? 8.0 : 4.0, ce = 2.0 * re;
    double by = 0.0, fl = 0.0;
    for (const int4& it : items) {
      const se::FftClass& c = ps.cls[it.x];
      const double in_b = kind == se::K_R2C ? c.n_in * re : (kind == se::K_C2R ? (c.n / 2 + 1) * ce : c.n_in * ce);
      const double out_b = kind == se::K_C2R ? c.n_out * re : c.n_out * ce;
      by += it.w * (in_b + out_b);
      fl += it.w * 5.0 * c.n * std::log2((double)c.n) * (kind == se::K_FUSED ? 2.0 : 1.0);
    }
    ps.alg_bytes = by;
    ps.alg_flops = fl;
  }
  if (ps.nitems == 0) {
    ps.items = nullptr;
    return true;
  }
  void* d = pl->dalloc(items.size() * sizeof(int4));
  if (!d) return false;
  if (hipMemcpy(d, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess) return false;
  ps.items = (const int4*)d;
  return true;
}

extern "C" {

const char* se_status_string(se_status s) {
  if ((int)s < 0 || (int)s >= (int)(sizeof(kStatusText) / sizeof(kStatusText[0]))) return "unknown status";
  return kStatusText[(int)s];
}

static bool valid_base(int D, double L, double xi, int M, int P) {
  if (D < 0 || D > 3) return false;
  if (!(L > 0) || !std::isfinite(L) || !(xi > 0) || !std::isfinite(xi)) return false;
  if (M < 2 || M % 2 || P < 2 || P % 2 || P > M || P > se::kMaxP) return false;
  return true;
}

static double fc(double x) {  // Eq. (fc-expression)
  return std::exp(-12.62 / (x * x)) * (0.8909 + 0.01411 * x + 4.315e-5 * x * x);
}

se_status se_params_default(int D, double L, double xi, int M, int P, se_window window, double Q,
                            double tol, se_precision prec, se_params* out) {
  if (!out) return SE_ERR_ARG;
  if (!valid_base(D, L, xi, M, P) || !(tol > 0) || !(Q >= 0)) return SE_ERR_PARAM;
  if (window != SE_WIN_GAUSSIAN && window != SE_WIN_PKB && window != SE_WIN_ES) return SE_ERR_PARAM;
  se_params p{};
  p.D = D;
  p.L = L;
  p.xi = xi;
  p.M = M;
  p.P = P;
  p.window = window;
  p.shape = window == SE_WIN_GAUSSIAN ? (kPi / 2.0) * P * 0.91 : 2.5 * P;
  p.nu = window == SE_WIN_PKB ? std::min(P / 2 + 2, 9) : 0;
  const double lam[2][3] = {{1.0, 1.5, 1.5}, {1.3, 2.4, 2.4}};  // Table lambda
  const double s0[3] = {2.8, 2.5, 2.0};
  p.lambda = D < 3 ? lam[window != SE_WIN_GAUSSIAN][D] : 0.0;
  p.s0 = D < 3 ? s0[D] : 0.0;
  p.tol = tol;
  p.Q = Q;
  p.prec = prec;
  p.s = 1.0;
  p.n_l = 0;
  if (D == 1 || D == 2) {
    const int Mt = smooth_even_up(2L * (long)std::ceil((M + p.lambda * P) / 2.0));
    const double B = std::sqrt(Q) * fc(xi * L) / L;  // Section 5.2
    const double lg = std::log(B / (2.0 * tol)) / (2.0 * kPi);
    p.s = std::max(1.0, (double)M / Mt * (1.0 + lg));                         // Eq. (estimate-s)
    p.n_l = (int)std::ceil((double)M / (Mt - M) * lg - 1.0);                  // Eq. (estimate-nl)
    p.n_l = std::max(0, std::min(M / 2, p.n_l));
  }
  p.tile = 0;
  *out = p;
  return SE_OK;
}

// Kolafa-Perram k-space truncation estimate, Eq. (KP_fourier_space), k_inf = M/2.
static double kp_kspace(double Q, double xi, double L, int M) {
  const double kinf = M / 2.0;
  return std::sqrt(Q) * xi / (kPi * kPi) * std::pow(kinf, -1.5) * std::exp(-std::pow(kPi * kinf / (xi * L), 2));
}

// Error-pollution bound f_W(x), Eq. (error_pollution).
static double pollution_fw(se_window w, double x) {  // ES: the KB bound
  return w == SE_WIN_GAUSSIAN ? x * x + 0.2 * x + 2.25 : 0.7 * x * x + 0.2 * x + 1.8;
}

se_status se_error_scale(double Q, double xi, double L, double* B) {
  if (!B) return SE_ERR_ARG;
  if (!(Q >= 0) || !(xi > 0) || !(L > 0) || !std::isfinite(Q) || !std::isfinite(xi) || !std::isfinite(L))
    return SE_ERR_PARAM;
  *B = std::sqrt(Q) * fc(xi * L) / L;
  return SE_OK;
}

// Principal branch of the Lambert W function, w e^w = x, for x >= 0: Halley's
// iteration from log(1 + x) (an upper bound of W(x) for x >= 0).
static double lambert_w0(double x) {
  double w = std::log1p(x);
  for (int it = 0; it < 64; ++it) {
    const double ew = std::exp(w), f = w * ew - x;
    const double d = ew * (w + 1.0) - (w + 2.0) * f / (2.0 * w + 2.0);
    const double nw = w - f / d;
    if (std::fabs(nw - w) <= 1e-15 * (1.0 + std::fabs(nw))) return nw;
    w = nw;
  }
  return w;
}

se_status se_rs_cutoff_for_tolerance(double L, double xi, double Q, double tol_rel, double* rc) {
  if (!rc) return SE_ERR_ARG;
  if (!(L > 0) || !(xi > 0) || !(Q > 0) || !(tol_rel > 0) || !std::isfinite(L) || !std::isfinite(xi) ||
      !std::isfinite(Q) || !std::isfinite(tol_rel))
    return SE_ERR_PARAM;
  // Eq. (KP_rc): the cutoff at which Eq. (KP_real_space) equals the absolute
  // tolerance eps = tol_rel B
  const double eps = tol_rel * std::sqrt(Q) * fc(xi * L) / L;
  const double arg = (4.0 / 3.0) * std::pow(Q / (xi * L * L * L * eps * eps), 2.0 / 3.0);
  *rc = std::sqrt(3.0) / (2.0 * xi) * std::sqrt(lambert_w0(arg));
  return SE_OK;
}

se_status se_params_recipe(int D, double L, double xi, double Q, double tol_rel, se_window window,
                           se_precision prec, se_params* out) {
  if (!out) return SE_ERR_ARG;
  if (D < 0 || D > 3 || !(L > 0) || !(xi > 0) || !(Q > 0) || !(tol_rel > 0) || !std::isfinite(L) ||
      !std::isfinite(xi) || !std::isfinite(Q) ||
      (window != SE_WIN_GAUSSIAN && window != SE_WIN_PKB && window != SE_WIN_ES))
    return SE_ERR_PARAM;
  const double B = std::sqrt(Q) * fc(xi * L) / L;
  const double eps = tol_rel * B;
  // Eq. (KP_kinf): k_inf = sqrt(3) xi L / (2 pi) sqrt(W(4/3 [Q / (pi xi L^3 eps^2)]^(2/3)))
  const double arg = 4.0 / 3.0 * std::pow(Q / (kPi * xi * L * L * L * eps * eps), 2.0 / 3.0);
  const double kinf = std::sqrt(3.0) * xi * L / (2.0 * kPi) * std::sqrt(lambert_w0(arg));
  if (!(2.0 * kinf < 4096.0)) return SE_ERR_PARAM;
  int M = smooth_even_up((long)std::ceil(2.0 * kinf - 1e-9));
  // window support from the approximation estimates (Section 5.2), rounded up to even
  const double Pr = window == SE_WIN_GAUSSIAN ? std::log(2.0 * B / eps) / ((kPi / 2.0) * std::sqrt(0.91))
                                              : std::log(10.0 * B / eps) / 2.5;
  int P = std::max(2, 2 * (int)std::ceil(Pr / 2.0 - 1e-12));
  // error pollution (Eq. error_pollution): 5 % more grid, P + 4
  if (P > pollution_fw(window, M / (xi * L))) {
    M = smooth_even_up((long)std::ceil(1.05 * M - 1e-9));
    P += 4;
  }
  if (P > se::kMaxP || M >= 4096) return SE_ERR_PARAM;
  M = std::max(M, smooth_even_up(P));
  return se_params_default(D, L, xi, M, P, window, Q, eps, prec, out);
}

se_status se_params_for_tolerance(int D, double L, double xi, double Q, double tol_rel, int P, se_window window,
                                  se_precision prec, se_params* out) {
  if (!out) return SE_ERR_ARG;
  if (D < 0 || D > 3 || !(L > 0) || !(xi > 0) || !(Q > 0) || !(tol_rel > 0) || P < 2 || P % 2 || P > se::kMaxP)
    return SE_ERR_PARAM;
  const double B = std::sqrt(Q) * fc(xi * L) / L;
  int M = std::max(P, 4);
  M = smooth_even_up(M);
  // smallest 7-smooth even M whose truncation estimate meets tol_rel * B,
  // then no error pollution: P <= f_W(M / (xi L))
  while (M < 4096 && (kp_kspace(Q, xi, L, M) > tol_rel * B || P > pollution_fw(window, M / (xi * L))))
    M = smooth_even_up(M + 2);
  if (M >= 4096) return SE_ERR_PARAM;
  return se_params_default(D, L, xi, M, P, window, Q, tol_rel * B, prec, out);
}

se_status se_plan_get_info(const se_plan* plan, se_plan_info* info) {
  if (!plan || !info) return SE_ERR_ARG;
  *info = plan->info;
  info->device_bytes = plan->bytes;
  return SE_OK;
}

se_status se_plan_destroy(se_plan* plan) {
  if (plan) {
    (void)hipSetDevice(plan->device);
    delete plan;
  }
  return SE_OK;
}

static se_status build_passes(se_plan* pl, hipStream_t st);
static void build_ik_passes(se_plan* pl);
static se_status precompute_0p(se_plan* pl, hipStream_t st, const void** table);

// Largest number of tile-box images (periodic copies included) that meet one
// tile in direction d; the fold kernel sums over at most kMaxFoldImages.
static int fold_image_count(const se::GridGeom& g, int d) {
  const int T = g.T[d], G = g.G[d], nt = g.nt[d], RX = T + g.P - 1, h = g.P / 2 - 1;
  int emin = T;
  if (g.per[d]) emin = std::min(T, G - (nt - 1) * T);
  const int reach = 2 + (T + g.P) / std::max(emin, 1);
  int most = 0;
  for (int t = 0; t < nt; ++t) {
    const int x0 = t * T, ext = std::min(T, G - x0);
    int n = 0;
    for (int dd = -reach; dd <= reach; ++dd) {
      int u = t + dd, shift = 0;
      if (!g.per[d] && (u < 0 || u >= nt)) continue;
      while (u < 0) u += nt, shift -= G;
      while (u >= nt) u -= nt, shift += G;
      const int o = u * T + shift - h;
      if (o < x0 + ext && o + RX > x0) ++n;
    }
    most = std::max(most, n);
  }
  return most;
}

// Clipped spreading: anchor pieces of one direction over all tiles (as the
// kernel forms them); returns the largest sub-bin count (sub-bins summed over
// pieces, or pieces when 'pieces_only'), or a value above every limit when a
// tile needs more than kMaxPieces pieces.
static int clip_dim_max(const se::GridGeom& g, int d, bool pieces_only) {
  const int T = g.T[d], G = g.G[d], nt = g.nt[d], h = g.P / 2;
  int most = 0;
  for (int t = 0; t < nt; ++t) {
    const int o = t * T, e = std::min(T, G - o);
    int lo = o - h, hi = o + e - 1 + h - 1, cnt = 0, np = 0;
    if (!g.per[d]) {
      lo = std::max(lo, 0);
      hi = std::min(hi, G - 1);
      if (lo <= hi) cnt = hi / se::kSB - lo / se::kSB + 1, np = 1;
    } else {
      auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((b - 1 - a) / b); };
      for (int k = fdiv(lo, G); k <= fdiv(hi, G); ++k) {
        const int a = std::max(lo - k * G, 0), b = std::min(hi - k * G, G - 1);
        if (a > b) continue;
        cnt += b / se::kSB - a / se::kSB + 1;
        ++np;
      }
    }
    if (np > se::kMaxPieces) return 1 << 28;
    most = std::max(most, pieces_only ? np : cnt);
  }
  return most;
}

static long clip_ranges_max(const se::GridGeom& g) {
  return (long)clip_dim_max(g, 2, false) * clip_dim_max(g, 1, false) * clip_dim_max(g, 0, true);
}

static se_status plan_create(const se_params* params, long n_max, void* hip_stream, size_t lds_soft,
                             long min_tiles, se_plan** out);

se_status se_plan_create(const se_params* params, long n_max, void* hip_stream, se_plan** out) {
  return plan_create(params, n_max, hip_stream, 65536, 512, out);
}

// lds_soft: LDS budget per workgroup that keeps several workgroups per CU;
// min_tiles: the automatic tile choice takes the largest tile shape that fits
// the budget and still gives at least this many tiles (a lone system needs
// many workgroups; a batch gets them from its other systems).
static se_status plan_create(const se_params* params, long n_max, void* hip_stream, size_t lds_soft,
                             long min_tiles, se_plan** out) {
  if (!params || !out || n_max < 0 || n_max > (1L << 30)) return SE_ERR_ARG;
  *out = nullptr;
  se_params p = *params;
  if (!valid_base(p.D, p.L, p.xi, p.M, p.P)) return SE_ERR_PARAM;
  if (p.window != SE_WIN_GAUSSIAN && p.window != SE_WIN_PKB && p.window != SE_WIN_ES) return SE_ERR_PARAM;
  if (p.deriv_fit < 0 || p.deriv_fit > 1 || (p.deriv_fit && p.window != SE_WIN_PKB)) return SE_ERR_PARAM;
  if (p.prec != SE_F64 && p.prec != SE_F32) return SE_ERR_PARAM;
  if (!is_smooth(p.M)) return SE_ERR_PARAM;
  // rectangular periodic cells: My, Mz grid intervals at spacing L/M in a
  // triply periodic box, My in a doubly periodic cell (z free, extent L)
  if (p.My <= 0) p.My = p.M;
  if (p.Mz <= 0) p.Mz = p.M;
  if (p.My != p.M || p.Mz != p.M) {
    if (p.D < 2 || (p.D == 2 && p.Mz != p.M)) return SE_ERR_PARAM;
    for (int m : {p.My, p.Mz})
      if (m % 2 || m < p.P || m > 4096 || !is_smooth(m)) return SE_ERR_PARAM;
  }
  if (!(p.shape > 0)) p.shape = p.window == SE_WIN_GAUSSIAN ? (kPi / 2.0) * p.P * 0.91 : 2.5 * p.P;
  if (p.window == SE_WIN_PKB) {
    if (p.nu <= 0) p.nu = std::min(p.P / 2 + 2, 9);
    if (p.nu > se::kMaxNu) return SE_ERR_PARAM;
  } else {
    p.nu = 0;
  }
  if (p.D < 3) {
    const double lam[2][3] = {{1.0, 1.5, 1.5}, {1.3, 2.4, 2.4}};
    const double s0[3] = {2.8, 2.5, 2.0};
    if (!(p.lambda > 0)) p.lambda = lam[p.window != SE_WIN_GAUSSIAN][p.D];
    if (!(p.s0 > 0)) p.s0 = s0[p.D];
    // Section 3.4: the zero mode (2P, 1P) and the free-space transform (0P)
    // need s0 >= 1 + sqrt(d) for d = 3 - D free directions
    if (p.lambda < 1.0 || p.s0 < 1.0 + std::sqrt((double)(3 - p.D)) - 1e-12) return SE_ERR_PARAM;
  }
  if (p.D == 1 || p.D == 2) {
    if (!(p.s > 0) || p.n_l < 0) {
      if (!(p.tol > 0) || !(p.Q > 0)) return SE_ERR_PARAM;
      se_params d;
      se_status s = se_params_default(p.D, p.L, p.xi, p.M, p.P, p.window, p.Q, p.tol, p.prec, &d);
      if (s != SE_OK) return s;
      if (!(p.s > 0)) p.s = d.s;
      if (p.n_l < 0) p.n_l = d.n_l;
    }
    if (p.s < 1.0) return SE_ERR_PARAM;
    p.n_l = std::min(p.n_l, p.M / 2);
  }

  se_plan* pl = new (std::nothrow) se_plan();
  if (!pl) return SE_ERR_NOMEM;
  pl->p = p;
  pl->f64 = (p.prec == SE_F64);
  pl->n_max = n_max;
  (void)hipGetDevice(&pl->device);
  pl->lds_limit = lds_soft;
  if (p.spread_mode < 0 || p.spread_mode > 3 || p.force_method < 0 || p.force_method > 2) {
    delete pl;
    return SE_ERR_PARAM;
  }
  if (p.fft_cap > 0) {
    if (p.fft_cap < 1024 || p.fft_cap > se::kFftCap || (p.fft_cap & (p.fft_cap - 1))) {
      delete pl;
      return SE_ERR_PARAM;
    }
    pl->fft_cap = p.fft_cap;
  }
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device) == hipSuccess && lds > 0)
    pl->lds_max = std::max<size_t>(pl->lds_limit, (size_t)lds);

  // ---- derived sizes, Algorithm 4 step 0 and Section 6 ----
  se_plan_info& I = pl->info;
  I.D = p.D;
  I.M = p.M;
  I.P = p.P;
  I.nu = p.nu;
  I.h = p.L / p.M;
  I.shape = p.shape;
  I.lambda = p.lambda;
  I.s0 = p.s0;
  I.s = p.s;
  I.n_l = (p.D == 1 || p.D == 2) ? p.n_l : 0;
  I.Mt = p.D == 3 ? p.M : smooth_even_up(2L * (long)std::ceil((p.M + p.lambda * p.P) / 2.0 - 1e-12));
  I.R = std::sqrt((double)(3 - p.D)) * I.h * I.Mt;
  I.n0 = p.D < 3 ? smooth_even_up((long)std::ceil(p.s0 * I.Mt - 1e-9)) : 0;
  I.nI = (p.D == 1 || p.D == 2) ? smooth_even_up((long)std::ceil(p.s * I.Mt - 1e-9)) : 0;
  for (int d = 0; d < 3; ++d) {
    const int Md = d == 0 ? p.M : (d == 1 ? p.My : p.Mz);   // periodic grid length (My = Mz = M below 3P)
    I.grid[d] = d < p.D ? Md : I.Mt;
    I.nfft[d] = d < p.D ? Md : (p.D == 0 ? 2 * I.Mt : I.Mt);
  }
  if (I.Mt >= 1024) {
    delete pl;
    return SE_ERR_PARAM;
  }

  // ---- geometry and tiles ----
  se::GridGeom& g = pl->geom;
  g.D = p.D;
  for (int d = 0; d < 3; ++d) {
    g.G[d] = I.grid[d];
    g.per[d] = d < p.D;
    g.d0[d] = d < p.D ? 0 : (I.Mt - p.M) / 2;
  }
  g.P = p.P;
  g.nu = p.nu;
  g.window = p.window == SE_WIN_PKB ? 1 : (p.window == SE_WIN_ES ? 2 : 0);
  g.h = I.h;
  g.L = p.L;
  for (int d = 0; d < 3; ++d) g.Lp[d] = I.grid[d] == p.M ? p.L : I.grid[d] * I.h;
  g.xi = p.xi;
  g.alpha = p.shape;
  g.scale = 4.0 * kPi * I.h * I.h * I.h;
  g.xcd = xcd_mode(p.xcd_tiles);
  // spreading mode: columns straight into the grid for sparse grids (fewer
  // than 0.05 particles per grid point), boxes and fold otherwise
  {
    const double npts = (double)I.grid[0] * I.grid[1] * I.grid[2];
    const bool sparse = (double)std::max(1L, n_max) < 0.05 * npts;
    const int mode = p.spread_mode > 0 ? p.spread_mode : (sparse ? 3 : 1);
    g.clip = mode - 1;
  }
  {
    // Largest tile whose spread and gather LDS fit, with at least min_tiles
    // tiles when the grid allows it.
    static const int cands[][3] = {{16, 16, 16}, {32, 16, 8}, {16, 16, 8}, {16, 8, 8}, {8, 8, 8},
                                   {8, 8, 4},    {8, 4, 4},   {4, 4, 4}};
    const bool explicit3 = p.tile3[0] > 0 && p.tile3[1] > 0 && p.tile3[2] > 0;
    if (explicit3)
      for (int d = 0; d < 3; ++d)
        if (p.tile3[d] % se::kSB || p.tile3[d] > 32) {
          delete pl;
          return SE_ERR_PARAM;
        }
    int best = -1, best_chunk = 64;
    for (size_t budget : {pl->lds_limit, pl->lds_max}) {
      for (int c = 0; c < (int)(sizeof(cands) / sizeof(cands[0])); ++c) {
        if (explicit3) {
          if (c > 0) break;
          for (int d = 0; d < 3; ++d) g.T[d] = p.tile3[d];
        } else {
          if (p.tile > 0 && !(cands[c][0] == p.tile && cands[c][1] == p.tile && cands[c][2] == p.tile)) continue;
          for (int d = 0; d < 3; ++d) g.T[d] = cands[c][d];
        }
        // column spreading: one thread per (x, y) column, at most kColZ points each
        if (g.clip == 2 && (g.T[0] * g.T[1] > se::kBlock || g.T[2] > se::kColZ)) {
          if (explicit3 || p.tile > 0) {
            delete pl;
            return SE_ERR_PARAM;
          }
          continue;
        }
        int fit = 0;
        for (int ch : {64, 32, 16}) {
          g.chunk = ch;
          if (se::spread_lds_bytes(g, pl->f64) <= budget && se::gather_lds_bytes(g, pl->f64) <= budget) {
            fit = ch;
            break;
          }
        }
        if (!fit) continue;
        long nt = 1;
        for (int d = 0; d < 3; ++d) nt *= (g.G[d] + g.T[d] - 1) / g.T[d];
        best = c;
        best_chunk = fit;
        if (explicit3 || p.tile > 0 || nt >= min_tiles) break;
      }
      if (best >= 0) break;
    }
    if (best < 0) {
      delete pl;
      return SE_ERR_UNSUPPORTED;
    }
    g.chunk = best_chunk;
    for (int d = 0; d < 3; ++d) g.T[d] = explicit3 ? p.tile3[d] : cands[best][d];
  }
  for (int d = 0; d < 3; ++d) I.tile[d] = g.T[d];
  I.fft_cap = pl->fft_cap > 0 ? pl->fft_cap : (pl->f64 ? 1024 : 2048);
  for (int d = 0; d < 3; ++d) {
    g.nt[d] = (g.G[d] + g.T[d] - 1) / g.T[d];
    g.nsb[d] = (g.G[d] + se::kSB - 1) / se::kSB;
  }
  pl->ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  if (g.clip && clip_ranges_max(g) > se::kMaxClipRanges) {
    if (p.spread_mode >= 2) {
      delete pl;
      return SE_ERR_UNSUPPORTED;
    }
    g.clip = 0;  // the automatic choice falls back to boxes and fold
    if (se::spread_lds_bytes(g, pl->f64) > pl->lds_max) {
      delete pl;
      return SE_ERR_UNSUPPORTED;
    }
  }
  I.spread_mode = g.clip + 1;
  if (!g.clip)
    for (int d = 0; d < 3; ++d)
      if (fold_image_count(g, d) > se::kMaxFoldImages) {
        delete pl;
        return SE_ERR_UNSUPPORTED;
      }
  pl->nsbtot = g.nsb[0] * g.nsb[1] * g.nsb[2];

  hipStream_t st = (hipStream_t)hip_stream;
  se_status rc = SE_OK;
  do {
    // ---- window table: coefficients and derivative coefficients ----
    const int m = p.nu + 1;
    std::vector<double> wt(2 * (size_t)p.P * m, 0.0);
    if (p.window == SE_WIN_PKB) {
      std::vector<double> c;
      if (!pkb_coefficients(p.P, p.shape, p.nu, c)) {
        rc = SE_ERR_PARAM;
        break;
      }
      std::vector<double> cd;
      if (p.deriv_fit && !pkb_coefficients(p.P, p.shape, p.nu, cd, kb_window_du)) {
        rc = SE_ERR_PARAM;
        break;
      }
      for (int i = 0; i < p.P; ++i)
        for (int j = 0; j < m; ++j) {
          wt[(size_t)i * m + j] = c[(size_t)i * m + j];
          if (p.deriv_fit)   // the fitted W'_KB(u), u = grid point minus particle: d/dx = -W'/h
            wt[(size_t)p.P * m + (size_t)i * m + j] = -cd[(size_t)i * m + j] / I.h;
          else if (j + 1 < m)   // d/dx of sum c_j xbar^j, xbar = 1 - 2 frac(x/h): chain factor -2/h
            wt[(size_t)p.P * m + (size_t)i * m + j] = (j + 1) * c[(size_t)i * m + j + 1] * (-2.0 / I.h);
        }
    }
    pl->buf.wtab = pl->upload(wt);
    if (!pl->buf.wtab) {
      rc = SE_ERR_NOMEM;
      break;
    }

    // ---- particle and tile buffers ----
    se::EvalBuffers& b = pl->buf;
    const size_t esz = pl->f64 ? 8 : 4;
    const long nm = std::max(1L, n_max);
    const int nblk = (int)((nm + se::kBlock - 1) / se::kBlock);
    // work buffers: laid out in the workspace (bound later by the caller)
    b.sb_count = (int*)pl->walloc(sizeof(int) * pl->nsbtot);
    b.sb_start = (int*)pl->walloc(sizeof(int) * (pl->nsbtot + 1));
    b.sb_cursor = (int*)pl->walloc(sizeof(int) * pl->nsbtot);
    b.p_key = (int*)pl->walloc(sizeof(int) * nm);
    b.p_cell = (int*)pl->walloc(sizeof(int) * nm);
    b.p_frac = pl->walloc(4 * esz * nm);
    b.s_cell = (int*)pl->walloc(sizeof(int) * nm);
    b.s_idx = (int*)pl->walloc(sizeof(int) * nm);
    b.s_fq = pl->walloc(4 * esz * nm);
    b.qpart = (double*)pl->walloc(sizeof(double) * 4 * nblk);
    b.bsum = (int*)pl->walloc(sizeof(int) * se::scan_blocks(g));
    b.stage = g.clip ? nullptr
                     : pl->walloc(esz * (size_t)pl->ntiles * (g.T[0] + p.P - 1) * (g.T[1] + p.P - 1) *
                                  (g.T[2] + p.P - 1));
    b.epart = (double*)pl->walloc(sizeof(double) * pl->ntiles);
    b.red = (double*)pl->walloc(sizeof(double) * 4);
    b.grid = pl->walloc(esz * (size_t)g.G[0] * g.G[1] * g.G[2]);
    b.vjp_phi = pl->walloc(esz * nm);
    b.vjp_grad = pl->walloc(3 * esz * nm);
    // the device status word persists across evaluations: plan-owned
    b.status = (int*)pl->dalloc(sizeof(int));
    if (!b.status) {
      rc = SE_ERR_NOMEM;
      break;
    }
    if (hipMemset(b.status, 0, sizeof(int)) != hipSuccess) {
      rc = SE_ERR_DEVICE;
      break;
    }
    rc = build_passes(pl, st);
    if (rc != SE_OK) break;
    if (p.force_method == 2) build_ik_passes(pl);
  } while (false);
  // table uploads are synchronous; the free-space precompute ran on st
  if (rc == SE_OK && hipStreamSynchronize(st) != hipSuccess) rc = SE_ERR_DEVICE;
  if (rc != SE_OK) {
    delete pl;
    return rc;
  }
  I.device_bytes = pl->bytes;
  I.workspace_bytes = pl->ws_bytes;
  I.fft_wide = 0;
  for (int k = 0; k < 5; ++k) I.fft_block[k] = 0;
  for (size_t k = 0; k < pl->passes.size(); ++k) {
    if (pl->passes[k].wide) I.fft_wide |= 1 << k;
    if (k < 5) I.fft_block[k] = pl->passes[k].B;
  }
  *out = pl;
  return SE_OK;
}

// Record the transform passes of Algorithm 4 steps 2-4 for this plan.
static se_status build_passes(se_plan* pl, hipStream_t st) {
  const se_params& p = pl->p;
  const se_plan_info& I = pl->info;
  const int D = p.D, M = p.M, Mt = I.Mt;
  const int Gx = I.grid[0], Gy = I.grid[1], Gz = I.grid[2];
  const size_t ce = pl->f64 ? 16 : 8;
  std::vector<std::vector<int>> rg;
  auto fail = [&]() { return SE_ERR_NOMEM; };
  // force method 2: signed-wavenumber tables and directions of a fused class
  const bool m2 = p.force_method == 2;
  bool dt_ok = true;
  auto set_d = [&](se::FftClass& c, int nA, int nB, int nC, int dirA, int dirB) {
    if (!m2) return;
    c.dA = pl->d_table(nA);
    c.dB = pl->d_table(nB);
    c.dC = pl->d_table(nC);
    c.dirA = dirA;
    c.dirB = dirB;
    dt_ok = dt_ok && c.dA && c.dB && c.dC;
  };

  if (D == 3 || D == 2) {
    const int nx = M, Kx = M / 2 + 1;
    void* cb = pl->walloc(ce * (size_t)Kx * Gy * Gz);
    pl->spec = {{(char*)cb, ce * (size_t)Kx * Gy * Gz}};
    const void* sepM = pl->sep_table(M);
    const void* k2M = pl->k2_table(M);
    if (!sepM || !k2M) return fail();
    // x: real-to-complex
    se::FftPass p1{};
    p1.cls[0] = make_class(nx, Gx, Kx, pl->buf.grid, cb, 1, Gx, (long long)Gx * Gy, 1, Kx, (long long)Kx * Gy);
    rg = {{0, 0, Gy, 0, Gz}};
    if (!finish_pass(pl, p1, se::K_R2C, 1, rg)) return fail();
    // y: complex forward (Gy = M, or My in a rectangular 3P box)
    se::FftPass p2{};
    p2.cls[0] = make_class(Gy, Gy, Gy, cb, cb, Kx, 1, (long long)Kx * Gy, Kx, 1, (long long)Kx * Gy);
    rg = {{0, 0, Kx, 0, Gz}};
    if (!finish_pass(pl, p2, se::K_C2C_FWD, 1, rg)) return fail();
    // z: fused forward / scale / inverse
    se::FftPass p3{};
    const long long zst = (long long)Kx * Gy;
    if (D == 3) {
      // z pencils of length Gz; the separable vectors and squared wavenumbers
      // of each direction come from its own transform length at spacing h
      // (all M in a cube)
      se::FftClass c = make_class(Gz, Gz, Gz, cb, cb, zst, 1, Kx, zst, 1, Kx);
      c.gmode = se::G_INVSQ;
      c.sA = sepM;
      c.sB = Gy == M ? sepM : pl->sep_table(Gy);
      c.sC = Gz == M ? sepM : pl->sep_table(Gz);
      c.kA = k2M;
      c.kB = Gy == M ? k2M : pl->k2_table(Gy);
      c.kC = Gz == M ? k2M : pl->k2_table(Gz);
      if (!c.sB || !c.sC || !c.kB || !c.kC) return fail();
      set_d(c, M, Gy, Gz, 0, 1);
      p3.cls[0] = c;
      rg = {{0, 0, Kx, 0, Gy}};
      if (!finish_pass(pl, p3, se::K_FUSED, 1, rg)) return fail();
    } else {
      // 2P: AFT classes, Algorithm 1 steps 2-4 / Algorithm 2 steps 1-3
      const int n0 = I.n0, nI = I.nI, nl = I.n_l;
      // y of length Gy (My in a rectangular cell, side Gy h): its own
      // separable vector and squared wavenumbers; the set I bounds the
      // wavenumber, index n_l along x and n_l Gy / M along y
      const int nly = (int)((long)nl * Gy / M);
      const void* sepY = Gy == M ? sepM : pl->sep_table(Gy);
      const void* k2Y = Gy == M ? k2M : pl->k2_table(Gy);
      const void* s0t = pl->sep_table(n0);
      const void* sIt = pl->sep_table(nI);
      const void* sJt = pl->sep_table(Mt);
      const void* kIt = pl->k2_table(nI);
      const void* kJt = pl->k2_table(Mt);
      if (!sepY || !k2Y) return fail();
      std::vector<double> g0(n0);
      for (int t = 0; t < n0; ++t) g0[t] = g2p_zero(2.0 * kPi * signed_freq(t, n0) / (n0 * I.h), I.R);
      const void* g0t = pl->upload(g0);
      if (!s0t || !sIt || !sJt || !kIt || !kJt || !g0t) return fail();
      se::FftClass c0 = make_class(n0, Mt, Mt, cb, cb, zst, 1, Kx, zst, 1, Kx);
      c0.gmode = se::G_TAB1;
      c0.sA = sepM;
      c0.sB = sepY;
      c0.sC = s0t;
      c0.gtab = g0t;
      se::FftClass cI = make_class(nI, Mt, Mt, cb, cb, zst, 1, Kx, zst, 1, Kx);
      cI.gmode = se::G_INVSQ;
      cI.sA = sepM;
      cI.sB = sepY;
      cI.kA = k2M;
      cI.kB = k2Y;
      cI.sC = sIt;
      cI.kC = kIt;
      se::FftClass cJ = make_class(Mt, Mt, Mt, cb, cb, zst, 1, Kx, zst, 1, Kx);
      cJ.gmode = se::G_INVSQ;
      cJ.sA = sepM;
      cJ.sB = sepY;
      cJ.kA = k2M;
      cJ.kB = k2Y;
      cJ.sC = sJt;
      cJ.kC = kJt;
      set_d(c0, M, Gy, n0, 0, 1);
      set_d(cI, M, Gy, nI, 0, 1);
      set_d(cJ, M, Gy, Mt, 0, 1);
      p3.cls[0] = c0;
      p3.cls[1] = cI;
      p3.cls[2] = cJ;
      rg.clear();
      for (int ky = 0; ky < Gy; ++ky) {
        const int sky = std::abs(signed_freq(ky, Gy) == Gy / 2 ? -Gy / 2 : signed_freq(ky, Gy));
        if (sky <= nly) {
          if (ky == 0) {
            rg.push_back({0, 0, 1, ky, ky + 1});
            if (nl >= 1) rg.push_back({1, 1, std::min(nl, Kx - 1) + 1, ky, ky + 1});
          } else {
            rg.push_back({1, 0, std::min(nl, Kx - 1) + 1, ky, ky + 1});
          }
          if (nl + 1 < Kx) rg.push_back({2, nl + 1, Kx, ky, ky + 1});
        } else {
          rg.push_back({2, 0, Kx, ky, ky + 1});
        }
      }
      if (!finish_pass(pl, p3, se::K_FUSED, 3, rg)) return fail();
    }
    se::FftPass p4 = p2;
    p4.kind = se::K_C2C_INV;
    se::FftPass p5{};
    p5.cls[0] = make_class(nx, Kx, Gx, cb, pl->buf.grid, 1, Kx, (long long)Kx * Gy, 1, Gx, (long long)Gx * Gy);
    rg = {{0, 0, Gy, 0, Gz}};
    if (!finish_pass(pl, p5, se::K_C2R, 1, rg)) return fail();
    pl->passes = {p1, p2, p3, p4, p5};
    return dt_ok ? SE_OK : fail();
  }

  if (D == 0) {
    const int n = 2 * Mt, Kx = Mt + 1;
    void* cb = pl->walloc(ce * (size_t)Kx * Mt * Mt);
    void* cb2 = pl->walloc(ce * (size_t)Kx * n * Mt);
    pl->spec = {{(char*)cb, ce * (size_t)Kx * Mt * Mt}, {(char*)cb2, ce * (size_t)Kx * n * Mt}};
    const void* sep = pl->sep_table(n);
    if (!sep) return fail();
    const void* table = nullptr;
    se_status rc = precompute_0p(pl, st, &table);
    if (rc != SE_OK) return rc;
    se::FftPass p1{};
    p1.cls[0] = make_class(n, Mt, Kx, pl->buf.grid, cb, 1, Mt, (long long)Mt * Mt, 1, Kx, (long long)Kx * Mt);
    rg = {{0, 0, Mt, 0, Mt}};
    if (!finish_pass(pl, p1, se::K_R2C, 1, rg)) return fail();
    se::FftPass p2{};
    p2.cls[0] = make_class(n, Mt, n, cb, cb2, Kx, 1, (long long)Kx * Mt, Kx, 1, (long long)Kx * n);
    rg = {{0, 0, Kx, 0, Mt}};
    if (!finish_pass(pl, p2, se::K_C2C_FWD, 1, rg)) return fail();
    se::FftPass p3{};
    const long long zst = (long long)Kx * n;
    se::FftClass c = make_class(n, Mt, Mt, cb2, cb2, zst, 1, Kx, zst, 1, Kx);
    c.gmode = se::G_TAB3;
    c.sA = c.sB = c.sC = sep;
    c.gtab = table;
    c.gd0 = c.gd1 = Mt + 1;
    c.fold0 = 0;
    c.fold1 = c.fold2 = n;
    set_d(c, n, n, n, 0, 1);
    p3.cls[0] = c;
    rg = {{0, 0, Kx, 0, n}};
    if (!finish_pass(pl, p3, se::K_FUSED, 1, rg)) return fail();
    se::FftPass p4{};
    p4.cls[0] = make_class(n, n, Mt, cb2, cb, Kx, 1, (long long)Kx * n, Kx, 1, (long long)Kx * Mt);
    rg = {{0, 0, Kx, 0, Mt}};
    if (!finish_pass(pl, p4, se::K_C2C_INV, 1, rg)) return fail();
    se::FftPass p5{};
    p5.cls[0] = make_class(n, Kx, Mt, cb, pl->buf.grid, 1, Kx, (long long)Kx * Mt, 1, Mt, (long long)Mt * Mt);
    rg = {{0, 0, Mt, 0, Mt}};
    if (!finish_pass(pl, p5, se::K_C2R, 1, rg)) return fail();
    pl->passes = {p1, p2, p3, p4, p5};
    return dt_ok ? SE_OK : fail();
  }

  // D == 1: periodic x, free y and z.  Classes over k_x: zero mode (n0),
  // set I = 1..n_l (nI), set J = n_l+1..M/2 (Mt).
  const int Kx = M / 2 + 1, n0 = I.n0, nI = I.nI;
  const int nl = std::min(I.n_l, Kx - 1);
  const int nJ = Kx - 1 - nl;
  void* cb = pl->walloc(ce * (size_t)Kx * Mt * Mt);
  void* b0 = pl->walloc(ce * (size_t)n0 * Mt);
  void* bI = pl->walloc(ce * (size_t)std::max(1, nl) * nI * Mt);
  pl->spec = {{(char*)cb, ce * (size_t)Kx * Mt * Mt}, {(char*)b0, ce * (size_t)n0 * Mt},
              {(char*)bI, ce * (size_t)std::max(1, nl) * nI * Mt}};
  const void* sepM = pl->sep_table(M);
  const void* k2M = pl->k2_table(M);
  const void* s0t = pl->sep_table(n0);
  const void* sIt = pl->sep_table(nI);
  const void* sJt = pl->sep_table(Mt);
  const void* kIt = pl->k2_table(nI);
  const void* kJt = pl->k2_table(Mt);
  const int h0 = n0 / 2 + 1;
  // zero-mode Green's function over the folded (k_z, k_y) frequencies, [k_z][k_y]
  std::vector<double> g1((size_t)h0 * h0);
  for (int iz = 0; iz < h0; ++iz)
    for (int iy = 0; iy < h0; ++iy) {
      const double ky = 2.0 * kPi * iy / (n0 * I.h), kz = 2.0 * kPi * iz / (n0 * I.h);
      g1[(size_t)iz * h0 + iy] = g1p_zero(std::sqrt(ky * ky + kz * kz), I.R);
    }
  const void* g1t = pl->upload(g1);
  if (!sepM || !k2M || !s0t || !sIt || !sJt || !kIt || !kJt || !g1t)
    return fail();
  char* cbc = (char*)cb;
  const long long mst = (long long)Kx * Mt;  // z stride of the main buffer
  // x: real-to-complex
  se::FftPass p1{};
  p1.cls[0] = make_class(M, Gx, Kx, pl->buf.grid, cb, 1, Gx, (long long)Gx * Gy, 1, Kx, mst);
  rg = {{0, 0, Gy, 0, Gz}};
  if (!finish_pass(pl, p1, se::K_R2C, 1, rg)) return fail();
  // y: padded forward transforms per class (Algorithm 1 steps 2-4, first free direction)
  se::FftPass p2{};
  p2.cls[0] = make_class(n0, Mt, n0, cb, b0, Kx, 0, mst, 1, 0, n0);
  p2.cls[1] = make_class(nI, Mt, nI, cbc + ce * 1, bI, Kx, 1, mst, nl, 1, (long long)nI * nl);
  p2.cls[2] = make_class(Mt, Mt, Mt, cbc + ce * (nl + 1), cbc + ce * (nl + 1), Kx, 1, mst, Kx, 1, mst);
  rg = {{0, 0, 1, 0, Mt}};
  if (nl > 0) rg.push_back({1, 0, nl, 0, Mt});
  if (nJ > 0) rg.push_back({2, 0, nJ, 0, Mt});
  if (!finish_pass(pl, p2, se::K_C2C_FWD, 3, rg)) return fail();
  // z: fused forward / scale / inverse per class
  se::FftPass p3{};
  {
    se::FftClass c0 = make_class(n0, Mt, Mt, b0, b0, n0, 1, 0, n0, 1, 0);
    c0.gmode = se::G_TAB2;
    c0.sA = s0t;
    c0.sB = sepM;
    c0.sC = s0t;
    c0.gtab = g1t;
    c0.gd0 = h0;
    c0.fold0 = n0;
    c0.fold2 = n0;
    se::FftClass cI = make_class(nI, Mt, Mt, bI, bI, (long long)nI * nl, 1, nl, (long long)nI * nl, 1, nl);
    cI.gmode = se::G_INVSQ;
    cI.sA = sepM;
    cI.kA = k2M;
    cI.offA = 1;
    cI.sB = sIt;
    cI.kB = kIt;
    cI.sC = sIt;
    cI.kC = kIt;
    se::FftClass cJ = make_class(Mt, Mt, Mt, cbc + ce * (nl + 1), cbc + ce * (nl + 1), mst, 1, Kx, mst, 1, Kx);
    cJ.gmode = se::G_INVSQ;
    cJ.sA = sepM;
    cJ.kA = k2M;
    cJ.offA = nl + 1;
    cJ.sB = sJt;
    cJ.kB = kJt;
    cJ.sC = sJt;
    cJ.kC = kJt;
    set_d(c0, n0, M, n0, 1, 0);   // b0: y on the zero mode's grid, b1: x (k_x = 0)
    set_d(cI, M, nI, nI, 0, 1);
    set_d(cJ, M, Mt, Mt, 0, 1);
    p3.cls[0] = c0;
    p3.cls[1] = cI;
    p3.cls[2] = cJ;
  }
  rg = {{0, 0, n0, 0, 1}};
  if (nl > 0) rg.push_back({1, 0, nl, 0, nI});
  if (nJ > 0) rg.push_back({2, 0, nJ, 0, Mt});
  if (!finish_pass(pl, p3, se::K_FUSED, 3, rg)) return fail();
  // y: inverse transforms with truncation back to Mt (Algorithm 2 steps 1-4)
  se::FftPass p4{};
  p4.cls[0] = make_class(n0, n0, Mt, b0, cb, 1, 0, n0, Kx, 0, mst);
  p4.cls[1] = make_class(nI, nI, Mt, bI, cbc + ce * 1, nl, 1, (long long)nI * nl, Kx, 1, mst);
  p4.cls[2] = p2.cls[2];
  rg = {{0, 0, 1, 0, Mt}};
  if (nl > 0) rg.push_back({1, 0, nl, 0, Mt});
  if (nJ > 0) rg.push_back({2, 0, nJ, 0, Mt});
  if (!finish_pass(pl, p4, se::K_C2C_INV, 3, rg)) return fail();
  // x: complex-to-real
  se::FftPass p5{};
  p5.cls[0] = make_class(M, Kx, Gx, cb, pl->buf.grid, 1, Kx, mst, 1, Gx, (long long)Gx * Gy);
  rg = {{0, 0, Gy, 0, Gz}};
  if (!finish_pass(pl, p5, se::K_C2R, 1, rg)) return fail();
  pl->passes = {p1, p2, p3, p4, p5};
  return dt_ok ? SE_OK : fail();
}

// Force method 2 (Section 7.2): per direction d, the fused pass with the
// factor i k_d reads the forward spectrum and writes shadow copies of the
// spectrum buffers, the inverse passes run on the shadows and the last one
// writes the grid, so the forward spectrum serves all three directions.
static void build_ik_passes(se_plan* pl) {
  std::vector<std::pair<char*, char*>> sh;   // (buffer, shadow)
  for (const auto& sb : pl->spec) sh.emplace_back(sb.first, (char*)pl->walloc(sb.second));
  auto map = [&](const void* ptr) -> void* {
    for (size_t k = 0; k < sh.size(); ++k) {
      const char* b = sh[k].first;
      if ((const char*)ptr >= b && (const char*)ptr < b + pl->spec[k].second)
        return sh[k].second + ((const char*)ptr - b);
    }
    return const_cast<void*>(ptr);
  };
  pl->ik_passes.clear();
  for (int d = 0; d < 3; ++d) {
    se::FftPass f = pl->passes[2], i4 = pl->passes[3], i5 = pl->passes[4];
    f.kind = se::K_FUSED_D;
    f.deriv = d;
    for (int c = 0; c < se::kMaxClasses; ++c) {
      f.cls[c].out = map(f.cls[c].out);
      i4.cls[c].in = map(i4.cls[c].in);
      i4.cls[c].out = map(i4.cls[c].out);
      i5.cls[c].in = map(i5.cls[c].in);
    }
    pl->ik_passes.push_back(f);
    pl->ik_passes.push_back(i4);
    pl->ik_passes.push_back(i5);
  }
}

// Algorithm 3 in FP64 on the GPU: sample G_hat^{0P} on the (s0 Mt)^3 grid,
// inverse transform, keep the offsets -Mt..Mt-1, forward transform, keep the
// real, even result as an octant table (Mt+1)^3 in the compute precision.
static se_status precompute_0p(se_plan* pl, hipStream_t st, const void** table) {
  const int Mt = pl->info.Mt, n0 = pl->info.n0, n = 2 * Mt;
  const double h = pl->info.h, R = pl->info.R;
  double* big = nullptr;
  double* small = nullptr;
  const size_t nb = (size_t)n0 * n0 * n0 * 16, ns = (size_t)n * n * n * 16;
  if (hipMalloc(&big, nb) != hipSuccess) return SE_ERR_NOMEM;
  if (hipMalloc(&small, ns) != hipSuccess) {
    (void)hipFree(big);
    return SE_ERR_NOMEM;
  }
  se_status rc = SE_OK;
  do {
    if (se::launch_g0p_fill(big, n0, h, R, st) != hipSuccess) {
      rc = SE_ERR_DEVICE;
      break;
    }
    // 3D complex transforms of an n^3 array: x (contiguous), y, z
    auto run3 = [&](double* a, int len, int kind) -> bool {
      const long long L1 = len, L2 = (long long)len * len;
      const long long st_[3] = {1, L1, L2}, s0_[3] = {L1, 1, 1}, s1_[3] = {L2, L2, L1};
      for (int ax = 0; ax < 3; ++ax) {
        se::FftPass ps{};
        ps.cls[0] = make_class(len, len, len, a, a, st_[ax], s0_[ax], s1_[ax], st_[ax], s0_[ax], s1_[ax]);
        const bool saved = pl->f64;
        pl->f64 = true;
        const bool ok = finish_pass(pl, ps, kind, 1, {{0, 0, len, 0, len}});
        pl->f64 = saved;
        if (!ok) return false;
        if (se::launch_fft(ps, true, st) != hipSuccess) return false;
      }
      return true;
    };
    if (!run3(big, n0, se::K_C2C_INV)) {
      rc = SE_ERR_DEVICE;
      break;
    }
    if (se::launch_g0p_truncate(big, n0, small, Mt, st) != hipSuccess) {
      rc = SE_ERR_DEVICE;
      break;
    }
    if (!run3(small, n, se::K_C2C_FWD)) {
      rc = SE_ERR_DEVICE;
      break;
    }
    const size_t esz = pl->f64 ? 8 : 4;
    void* tab = pl->dalloc(esz * (size_t)(Mt + 1) * (Mt + 1) * (Mt + 1));
    if (!tab) {
      rc = SE_ERR_NOMEM;
      break;
    }
    if (se::launch_g0p_fold(small, Mt, tab, pl->f64, st) != hipSuccess) {
      rc = SE_ERR_DEVICE;
      break;
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
      rc = SE_ERR_DEVICE;
      break;
    }
    *table = tab;
  } while (false);
  (void)hipFree(big);
  (void)hipFree(small);
  return rc;
}

namespace {
const char* kFftNames[] = {"fft_c2c_fwd", "fft_c2c_inv", "fft_r2c", "fft_c2r", "fft_fused_scale"};
constexpr int kEventPool = 8192;
}  // namespace

static se_status eval_bound(se_plan* plan, long N, const void* xyz, const void* q, void* phi, void* force,
                            double* energy, unsigned flags, void* hip_stream, int method);

se_status se_plan_workspace_size(const se_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return SE_ERR_ARG;
  *bytes = plan->ws_bytes;
  return SE_OK;
}

se_status se_plan_set_workspace(se_plan* plan, void* ptr, size_t bytes) {
  if (!plan) return SE_ERR_ARG;
  if (!ptr) {
    plan->rebase(kWsStandIn);
    plan->ws_bound = false;
    return SE_OK;
  }
  if (((uintptr_t)ptr & 255) || bytes < plan->ws_bytes) return SE_ERR_WORKSPACE;
  plan->rebase((uintptr_t)ptr);
  plan->ws_bound = true;
  return SE_OK;
}

se_status se_eval(se_plan* plan, long N, const void* xyz, const void* q, void* phi, void* force,
                  double* energy, unsigned flags, void* hip_stream) {
  if (!plan || N < 0 || N > plan->n_max) return SE_ERR_ARG;
  if (N > 0 && (!xyz || !q)) return SE_ERR_ARG;
  if (flags & ~(SE_IN_F32 | SE_ADD_SELF | SE_SYNC_CHECK | SE_OUT_GRAD | SE_ALLOW_NONNEUTRAL | SE_PROFILE))
    return SE_ERR_ARG;
  if (!plan->ws_bound) return SE_ERR_WORKSPACE;
  return eval_bound(plan, N, xyz, q, phi, force, energy, flags, hip_stream, plan->p.force_method);
}

// se_eval on a plan whose work pointers point at a workspace; forces by
// method 'method' (2: i k in the scaling step, else the window gradient).
static se_status eval_bound(se_plan* plan, long N, const void* xyz, const void* q, void* phi, void* force,
                            double* energy, unsigned flags, void* hip_stream, int method) {
  hipStream_t st = (hipStream_t)hip_stream;
  const se::GridGeom& g = plan->geom;
  se::EvalBuffers& b = plan->buf;
  const bool f64 = plan->f64;
  const int nblk = (int)((N + se::kBlock - 1) / se::kBlock);
  const double self_coef = (flags & SE_ADD_SELF) ? -2.0 * plan->p.xi / std::sqrt(kPi) : 0.0;

  // tracing: an event pair around each launch site
  const bool prof = (flags & SE_PROFILE) != 0;
  if (prof && plan->evpool.empty()) {
    plan->evpool.resize(kEventPool);
    for (auto& e : plan->evpool)
      if (hipEventCreate(&e) != hipSuccess) return SE_ERR_DEVICE;
  }
  int cur = -1;
  auto begin = [&]() {
    cur = -1;
    if (prof && plan->ev_used + 2 <= (int)plan->evpool.size()) {
      cur = plan->ev_used;
      plan->ev_used += 2;
      (void)hipEventRecord(plan->evpool[cur], st);
    }
  };
  auto end = [&](int site, double bytes, double flops) {
    if (cur >= 0) {
      (void)hipEventRecord(plan->evpool[cur + 1], st);
      plan->prof.push_back({site, cur, bytes, flops});
    }
  };
  const double re = f64 ? 8.0 : 4.0;
  const double in_e = (flags & SE_IN_F32) ? 4.0 : 8.0;
  const double G = (double)g.G[0] * g.G[1] * g.G[2];
  const int P = g.P, nu = std::max(g.nu, 5);

  begin();
  if (se::launch_zero(g, b, st) != hipSuccess) return SE_ERR_DEVICE;
  if (se::launch_bin(g, b, N, xyz, q, (flags & SE_IN_F32) != 0, f64, nblk, st) != hipSuccess) return SE_ERR_DEVICE;
  end(0, N * 4.0 * in_e, 0.0);
  begin();
  if (se::launch_scan(g, b, nblk, plan->p.D >= 1 && !(flags & SE_ALLOW_NONNEUTRAL), st) != hipSuccess)
    return SE_ERR_DEVICE;
  end(1, plan->nsbtot * 12.0, 0.0);
  begin();
  if (se::launch_scatter(g, b, N, f64, st) != hipSuccess) return SE_ERR_DEVICE;
  // sub-bins in input order: the column sums and the per-tile energy partials
  // then add in an order that does not depend on the scatter's atomics
  if (se::launch_order(g, b, plan->nsbtot, f64, st) != hipSuccess) return SE_ERR_DEVICE;
  end(2, N * 2.0 * (8.0 + 4.0 * re), 0.0);
  begin();
  if (se::launch_spread(g, b, f64, st) != hipSuccess) return SE_ERR_DEVICE;
  end(3, N * 4.0 * re + G * re, N * 2.0 * (3.0 * P * nu + P * P + (double)P * P * P));
  if (!g.clip) {
    begin();
    if (se::launch_fold(g, b, f64, st) != hipSuccess) return SE_ERR_DEVICE;
    const double R3 = (double)(g.T[0] + P - 1) * (g.T[1] + P - 1) * (g.T[2] + P - 1);
    end(4, plan->ntiles * R3 * re + G * re, plan->ntiles * R3);
  }
  const int np = (int)plan->passes.size();
  const int s_gather = 5 + np;
  auto run_pass = [&](const se::FftPass& ps, int site) -> bool {
    begin();
    if (se::launch_fft(ps, f64, st) != hipSuccess) return false;
    end(site, ps.alg_bytes, ps.alg_flops);
    return true;
  };
  const int og = (flags & SE_OUT_GRAD) ? 1 : 0;
  // a gathering of values only (method 2 and the potential without forces)
  const double val_bytes = N * 5.0 * re + G * re, val_flops = N * 2.0 * (3.0 * P * nu + P * P + (double)P * P * P);
  if (method == 2 && force && plan->ik_passes.size() == 9) {
    // force method 2 (Section 7.2): forward transforms once, then per
    // direction d the scaling with i k_d, the inverse transforms and a
    // gathering with the window itself into force column d
    for (int i = 0; i < 2; ++i)
      if (!run_pass(plan->passes[i], 5 + i)) return SE_ERR_DEVICE;
    for (int d = 0; d < 3; ++d) {
      for (int k = 0; k < 3; ++k)
        if (!run_pass(plan->ik_passes[3 * d + k], k == 0 ? s_gather + 2 : s_gather + 3)) return SE_ERR_DEVICE;
      begin();
      if (se::launch_gather(g, b, f64, nullptr, force, og, 0.0, st, se::GM_COMP, d) != hipSuccess)
        return SE_ERR_DEVICE;
      end(s_gather + 4, val_bytes, val_flops);
    }
    // the potential (and the energy) from the plain scaling, last: the fused
    // pass transforms the forward spectrum in place
    if (phi || energy) {
      for (int i = 2; i < np; ++i)
        if (!run_pass(plan->passes[i], 5 + i)) return SE_ERR_DEVICE;
      begin();
      if (se::launch_gather(g, b, f64, phi, nullptr, og, self_coef, st, se::GM_PHI) != hipSuccess)
        return SE_ERR_DEVICE;
      end(s_gather, val_bytes, val_flops);
    }
  } else {
    for (int i = 0; i < np; ++i)
      if (!run_pass(plan->passes[i], 5 + i)) return SE_ERR_DEVICE;
    if (phi || force || energy) {
      begin();
      const bool grad = force != nullptr;
      if (se::launch_gather(g, b, f64, phi, force, og, self_coef, st, grad ? se::GM_ALL : se::GM_PHI) !=
          hipSuccess)
        return SE_ERR_DEVICE;
      if (grad)
        end(s_gather, N * 8.0 * re + G * re, N * 2.0 * (6.0 * P * nu + 3.0 * P * P + (double)P * P * (2 * P + 4)));
      else
        end(s_gather, val_bytes, val_flops);
    }
  }
  if (energy) {
    begin();
    if (se::launch_energy(g, b, energy, 0.0, st) != hipSuccess) return SE_ERR_DEVICE;
    end(s_gather + 1, plan->ntiles * 8.0 + 8.0, 0.0);
  }
  if (flags & SE_SYNC_CHECK) return se_get_device_status(plan, hip_stream);
  return SE_OK;
}

se_status se_plan_profile(se_plan* plan, void* hip_stream, se_stage_record* out, int cap, int* n,
                          int reset) {
  if (!plan || !n || (cap > 0 && !out)) return SE_ERR_ARG;
  if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return SE_ERR_DEVICE;
  const int nsites = 10 + (int)plan->passes.size();
  std::vector<se_stage_record> agg(nsites);
  std::vector<double> bsum(nsites, 0.0), fsum(nsites, 0.0);
  for (int s = 0; s < nsites; ++s) {
    se_stage_record& r = agg[s];
    std::memset(&r, 0, sizeof(r));
    const char* nm;
    char buf[32];
    if (s == 0) nm = "bin";
    else if (s == 1) nm = "scan";
    else if (s == 2) nm = "scatter";
    else if (s == 3) nm = "spread";
    else if (s == 4) nm = "fold";
    else if (s < 5 + (int)plan->passes.size()) {
      std::snprintf(buf, sizeof(buf), "%s_%d", kFftNames[plan->passes[s - 5].kind], s - 4);
      nm = buf;
    } else if (s == 5 + (int)plan->passes.size()) nm = "gather";
    else if (s == 6 + (int)plan->passes.size()) nm = "energy";
    else if (s == 7 + (int)plan->passes.size()) nm = "ik_fused";
    else if (s == 8 + (int)plan->passes.size()) nm = "ik_inverse";
    else nm = "ik_gather";
    std::snprintf(r.name, sizeof(r.name), "%s", nm);
  }
  for (const auto& rec : plan->prof) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, plan->evpool[rec.ev], plan->evpool[rec.ev + 1]) != hipSuccess)
      return SE_ERR_DEVICE;
    se_stage_record& r = agg[rec.site];
    r.launches += 1;
    r.ms_total += ms;
    bsum[rec.site] += rec.bytes;
    fsum[rec.site] += rec.flops;
  }
  int k = 0;
  for (int s = 0; s < nsites; ++s) {
    if (agg[s].launches == 0) continue;
    agg[s].bytes = bsum[s] / agg[s].launches;
    agg[s].flops = fsum[s] / agg[s].launches;
    if (k < cap) out[k] = agg[s];
    ++k;
  }
  *n = std::min(k, cap);
  if (reset) {
    plan->prof.clear();
    plan->ev_used = 0;
  }
  return SE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Evaluation without allocation: the workspace is a static device array of
// SE_STATIC_SCRATCH_BYTES, one copy per device for the life of the process.
// Host code never passes the array's name to a kernel (on the host it is
// only a stand-in); it uses the device address hipGetSymbolAddress returns
// for the current device, looked up once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SE_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's copy of the scratch array.
se_status scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SE_ERR_DEVICE;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return SE_OK;
}
}  // namespace

extern "C" {

se_status se_eval_static(se_plan* plan, long N, const void* xyz, const void* q, void* phi, void* force,
                         double* energy, unsigned flags, void* hip_stream) {
  if (!plan || N < 0 || N > plan->n_max) return SE_ERR_ARG;
  if (N > 0 && (!xyz || !q)) return SE_ERR_ARG;
  // SE_PROFILE is refused: its event pool is created on first use
  if (flags & ~(SE_IN_F32 | SE_ADD_SELF | SE_SYNC_CHECK | SE_OUT_GRAD | SE_ALLOW_NONNEUTRAL)) return SE_ERR_ARG;
  if (plan->ws_bytes > SE_STATIC_SCRATCH_BYTES) return SE_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SE_ERR_DEVICE;
  if (dev != plan->device) return SE_ERR_ARG;
  if (dev < 0 || dev >= kMaxScratchDevices) return SE_ERR_UNSUPPORTED;
  void* base = nullptr;
  const se_status sa = scratch_address(dev, &base);
  if (sa != SE_OK) return sa;
  // point the plan's work buffers at the scratch for this call only; the
  // kernels receive them by value, so the caller's binding returns at once
  const uintptr_t prev = plan->ws_base;
  const bool prev_bound = plan->ws_bound;
  plan->rebase((uintptr_t)base);
  const se_status rc = eval_bound(plan, N, xyz, q, phi, force, energy, flags, hip_stream, plan->p.force_method);
  plan->rebase(prev);
  plan->ws_bound = prev_bound;
  return rc;
}

se_status se_get_device_status(se_plan* plan, void* hip_stream) {
  if (!plan) return SE_ERR_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  int s = 0;
  if (hipStreamSynchronize(st) != hipSuccess) return SE_ERR_DEVICE;
  if (hipMemcpy(&s, plan->buf.status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SE_ERR_DEVICE;
  if (s && hipMemset(plan->buf.status, 0, sizeof(int)) != hipSuccess) return SE_ERR_DEVICE;
  if (s & 1) return SE_ERR_NONFINITE;
  if (s & 2) return SE_ERR_OUT_OF_BOX;
  if (s & 4) return SE_ERR_NONNEUTRAL;
  return SE_OK;
}

se_status se_eval_vjp(se_plan* plan, long N, const void* xyz, const void* q, const void* g, const void* grad_phi,
                      void* grad_x, void* grad_q, unsigned flags, void* hip_stream) {
  if (!plan || N < 0 || N > plan->n_max) return SE_ERR_ARG;
  if (N > 0 && (!xyz || !q || !g || (grad_x && !grad_phi))) return SE_ERR_ARG;
  if (flags & ~(SE_IN_F32 | SE_ADD_SELF | SE_SYNC_CHECK)) return SE_ERR_ARG;
  if (!plan->ws_bound) return SE_ERR_WORKSPACE;
  if (!grad_x && !grad_q) return SE_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  // Algorithm 4 with the cotangent as charges: A g and grad (A g)
  const unsigned ef = (flags & (SE_IN_F32 | SE_ADD_SELF)) | SE_OUT_GRAD | SE_ALLOW_NONNEUTRAL;
  // method 1: the exact gradient of the discrete operator, which the
  // symmetry argument above needs
  se_status rc = eval_bound(plan, N, xyz, g, plan->buf.vjp_phi, grad_x ? plan->buf.vjp_grad : nullptr, nullptr,
                            ef, hip_stream, 1);
  if (rc != SE_OK) return rc;
  if (se::launch_potential_vjp(N, (flags & SE_IN_F32) != 0, plan->f64, q, g, grad_phi, plan->buf.vjp_phi,
                               plan->buf.vjp_grad, grad_x, grad_q, st) != hipSuccess)
    return SE_ERR_DEVICE;
  if (flags & SE_SYNC_CHECK) return se_get_device_status(plan, hip_stream);
  return SE_OK;
}

se_status se_energy_vjp(long N, se_precision prec, const double* grad_E, const void* q, const void* phi,
                        const void* grad_phi, void* grad_x, void* grad_q, unsigned flags, void* hip_stream) {
  if (N < 0 || (prec != SE_F64 && prec != SE_F32) || (flags & ~SE_IN_F32)) return SE_ERR_ARG;
  if (N > 0 && (!grad_E || (grad_x && (!q || !grad_phi)) || (grad_q && !phi))) return SE_ERR_ARG;
  if (se::launch_energy_vjp(N, (flags & SE_IN_F32) != 0, prec == SE_F64, grad_E, q, phi, grad_phi, grad_x, grad_q,
                            (hipStream_t)hip_stream) != hipSuccess)
    return SE_ERR_DEVICE;
  return SE_OK;
}

// ---------------------------------------------------------------------------
// Batched plans: one sub-plan per system; one launch per stage of the path
// over the work items of all systems.
// ---------------------------------------------------------------------------
}  // extern "C"

struct se_batch_plan {
  std::vector<se_plan*> sys;
  std::vector<long> N, off;
  long total = 0;
  se::SysDesc* d_sys = nullptr;
  int* d_off = nullptr;
  int4* d_rec = nullptr;                        // transform work records, list by list
  int items[se::BL_COUNT] = {};                // work items per list
  size_t lds[se::BS_COUNT] = {};               // dynamic LDS per stage launch
  int P = 0;
  bool f64 = true;
  int device = 0;
  // workspace: the sub-plans' workspaces one after another (256-byte aligned)
  std::vector<se::SysDesc> desc;
  std::vector<size_t> ws_off;
  size_t ws_bytes = 0;
  bool ws_bound = false;
  // algorithmic counts of one evaluation per stage, summed over systems
  double st_bytes[se::BS_COUNT] = {}, st_flops[se::BS_COUNT] = {};
  hipEvent_t ev[se::BS_COUNT + 1] = {};
  bool have_ev = false;
  int prof_pending = 0, prof_launches = 0;
  double st_ms[se::BS_COUNT] = {};
  ~se_batch_plan() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (d_sys) (void)hipFree(d_sys);
    if (d_off) (void)hipFree(d_off);
    if (d_rec) (void)hipFree(d_rec);
    for (se_plan* s : sys) delete s;
  }
  // fold the timings of the last profiled evaluation in (events complete)
  se_status collect() {
    if (!prof_pending) return SE_OK;
    if (hipEventSynchronize(ev[se::BS_COUNT]) != hipSuccess) return SE_ERR_DEVICE;
    for (int k = 0; k < se::BS_COUNT; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) return SE_ERR_DEVICE;
      st_ms[k] += ms;
    }
    prof_launches += 1;
    prof_pending = 0;
    return SE_OK;
  }
};

static const char* const kBatchStageNames[se::BS_COUNT] = {
    "zero", "bin", "scan1", "scan2", "scatter", "order", "spread", "fold",
    "fft0", "fft1", "fft2", "fft3", "fft4", "gather", "energy"};

extern "C" {

se_status se_batch_plan_create(const se_params* params, const long* N, int n_sys, void* hip_stream,
                               se_batch_plan** out) {
  if (!params || !N || !out || n_sys < 1) return SE_ERR_ARG;
  *out = nullptr;
  for (int s = 0; s < n_sys; ++s) {
    if (N[s] < 0) return SE_ERR_ARG;
    if (params[s].P != params[0].P || params[s].window != params[0].window || params[s].prec != params[0].prec ||
        params[s].force_method == 2)
      return SE_ERR_UNSUPPORTED;
  }
  const int P = params[0].P;
  if (P != 4 && P != 6 && P != 8 && P != 10 && P != 12) return SE_ERR_UNSUPPORTED;
  se_batch_plan* bp = new (std::nothrow) se_batch_plan();
  if (!bp) return SE_ERR_NOMEM;
  bp->P = P;
  bp->f64 = params[0].prec == SE_F64;
  (void)hipGetDevice(&bp->device);
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<se::SysDesc> desc(n_sys);
  std::vector<int> off((size_t)se::BL_COUNT * (n_sys + 1), 0);
  std::vector<std::vector<int4>> lrec((size_t)se::kPasses * se::kFftKinds);   // per transform list
  long run = 0;
  for (int s = 0; s < n_sys; ++s) {
    se_plan* sp = nullptr;
    se_status rc = plan_create(&params[s], N[s], hip_stream, 64 * 1024, 1, &sp);
    if (rc != SE_OK) {
      delete bp;
      return rc;
    }
    bp->sys.push_back(sp);
    if (sp->passes.size() != (size_t)se::kPasses) {
      delete bp;
      return SE_ERR_UNSUPPORTED;
    }
    se::SysDesc& d = desc[s];
    std::memset(&d, 0, sizeof(d));
    d.g = sp->geom;
    d.b = sp->buf;
    for (int k = 0; k < se::kPasses; ++k) d.pass[k] = sp->passes[k];
    d.N = N[s];
    d.off = run;
    d.nblk_bin = (int)((N[s] + se::kBlock - 1) / se::kBlock);
    d.nscan = se::scan_blocks(sp->geom);
    d.ntiles = sp->ntiles;
    d.check_neutral = sp->p.D >= 1;
    d.self_coef = -2.0 * sp->p.xi / std::sqrt(kPi);
    bp->N.push_back(N[s]);
    bp->off.push_back(run);
    run += N[s];
    const int n_order = (sp->nsbtot + se::kBlock - 1) / se::kBlock;
    const int items[se::BS_COUNT] = {d.nscan, d.nblk_bin, d.nscan, d.nscan, d.nblk_bin, n_order, d.ntiles,
                                     d.g.clip ? 0 : d.ntiles,
                                     d.pass[0].nitems, d.pass[1].nitems, d.pass[2].nitems, d.pass[3].nitems,
                                     d.pass[4].nitems, d.ntiles, 1};
    for (int k = 0; k < se::BS_COUNT; ++k) off[(size_t)k * (n_sys + 1) + s + 1] = items[k];
    for (int k = 0; k < se::kPasses; ++k) {
      off[(size_t)se::fft_list(se::BS_FFT0 + k, d.pass[k].kind) * (n_sys + 1) + s + 1] = d.pass[k].nitems;
      // this system's records of transform list (stage k, kind): {s * 4 + class, b0, b1, count}
      std::vector<int4> it(d.pass[k].nitems);
      if (!it.empty() && hipMemcpy(it.data(), d.pass[k].items, it.size() * sizeof(int4), hipMemcpyDeviceToHost) !=
                             hipSuccess) {
        delete bp;
        return SE_ERR_DEVICE;
      }
      auto& dst = lrec[(size_t)k * se::kFftKinds + d.pass[k].kind];
      for (const int4& r : it) dst.push_back(make_int4(s * 4 + r.x, r.y, r.z, r.w));
    }
    size_t* lds = bp->lds;
    lds[se::BS_SPREAD] = std::max(lds[se::BS_SPREAD], se::spread_lds_bytes(sp->geom, bp->f64));
    lds[se::BS_GATHER] = std::max(lds[se::BS_GATHER], se::gather_lds_bytes(sp->geom, bp->f64));
    for (int k = 0; k < se::kPasses; ++k)
      lds[se::BS_FFT0 + k] = std::max(lds[se::BS_FFT0 + k], se::fft_lds_bytes(d.pass[k], bp->f64));
    // algorithmic counts of one evaluation of this system, per stage (as for se_eval)
    const double re = bp->f64 ? 8.0 : 4.0;
    const double G = (double)d.g.G[0] * d.g.G[1] * d.g.G[2];
    const double R3 = (double)(d.g.T[0] + P - 1) * (d.g.T[1] + P - 1) * (d.g.T[2] + P - 1);
    const int nu = std::max(d.g.nu, 5);
    const double n = (double)N[s];
    double* by = bp->st_bytes;
    double* fl = bp->st_flops;
    by[se::BS_ZERO] += sp->nsbtot * 4.0;
    by[se::BS_BIN] += n * 4.0 * re;
    by[se::BS_SCAN1] += sp->nsbtot * 8.0;
    by[se::BS_SCAN2] += sp->nsbtot * 8.0;
    by[se::BS_SCATTER] += n * 2.0 * (8.0 + 4.0 * re);
    if (n_order) by[se::BS_ORDER] += n * 2.0 * (8.0 + 4.0 * re);
    by[se::BS_SPREAD] += n * 4.0 * re + G * re;
    fl[se::BS_SPREAD] += n * 2.0 * (3.0 * P * nu + P * P + (double)P * P * P);
    if (!d.g.clip) {
      by[se::BS_FOLD] += d.ntiles * R3 * re + G * re;
      fl[se::BS_FOLD] += d.ntiles * R3;
    }
    for (int k = 0; k < se::kPasses; ++k) {
      by[se::BS_FFT0 + k] += d.pass[k].alg_bytes;
      fl[se::BS_FFT0 + k] += d.pass[k].alg_flops;
    }
    by[se::BS_GATHER] += n * 8.0 * re + G * re;
    fl[se::BS_GATHER] += n * 2.0 * (6.0 * P * nu + 3.0 * P * P + (double)P * P * (2 * P + 4));
    by[se::BS_ENERGY] += d.ntiles * 8.0 + 8.0;
  }
  bp->total = run;
  for (se_plan* sp : bp->sys) {
    bp->ws_off.push_back(bp->ws_bytes);
    bp->ws_bytes += (sp->ws_bytes + 255) & ~(size_t)255;
  }
  for (int k = 0; k < se::BL_COUNT; ++k)
    for (int s = 0; s < n_sys; ++s) off[(size_t)k * (n_sys + 1) + s + 1] += off[(size_t)k * (n_sys + 1) + s];
  int lds_max = 0;
  (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, bp->device);
  if (lds_max > 0 && *std::max_element(bp->lds, bp->lds + se::BS_COUNT) > (size_t)lds_max) {
    delete bp;
    return SE_ERR_UNSUPPORTED;
  }
  for (int k = 0; k < se::BL_COUNT; ++k) bp->items[k] = off[(size_t)k * (n_sys + 1) + n_sys];
  if (hipMalloc(&bp->d_sys, sizeof(se::SysDesc) * n_sys) != hipSuccess ||
      hipMalloc(&bp->d_off, sizeof(int) * off.size()) != hipSuccess) {
    delete bp;
    return SE_ERR_NOMEM;
  }
  std::vector<int4> rec;
  for (const auto& l : lrec) rec.insert(rec.end(), l.begin(), l.end());
  if (hipMalloc(&bp->d_rec, sizeof(int4) * std::max<size_t>(rec.size(), 1)) != hipSuccess) {
    delete bp;
    return SE_ERR_NOMEM;
  }
  bp->desc = desc;
  if (hipMemcpy(bp->d_sys, desc.data(), sizeof(se::SysDesc) * n_sys, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(bp->d_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice) != hipSuccess ||
      (!rec.empty() && hipMemcpy(bp->d_rec, rec.data(), sizeof(int4) * rec.size(), hipMemcpyHostToDevice) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess) {
    delete bp;
    return SE_ERR_DEVICE;
  }
  *out = bp;
  return SE_OK;
}

se_status se_batch_plan_get_info(const se_batch_plan* plan, int sys, se_plan_info* info, long* n_particles,
                                 int* persistent_blocks) {
  // persistent_blocks is the 'reserved' output of the header
  if (!plan || sys < 0 || sys >= (int)plan->sys.size()) return SE_ERR_ARG;
  if (info) {
    *info = plan->sys[sys]->info;
    info->device_bytes = plan->sys[sys]->bytes;
    info->workspace_bytes = plan->sys[sys]->ws_bytes;
  }
  if (n_particles) *n_particles = plan->N[sys];
  if (persistent_blocks) *persistent_blocks = 0;
  return SE_OK;
}

se_status se_batch_plan_workspace_size(const se_batch_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return SE_ERR_ARG;
  *bytes = plan->ws_bytes;
  return SE_OK;
}

se_status se_batch_plan_set_workspace(se_batch_plan* plan, void* ptr, size_t bytes) {
  if (!plan) return SE_ERR_ARG;
  if (ptr && (((uintptr_t)ptr & 255) || bytes < plan->ws_bytes)) return SE_ERR_WORKSPACE;
  for (size_t s = 0; s < plan->sys.size(); ++s) {
    se_plan* sp = plan->sys[s];
    sp->rebase(ptr ? (uintptr_t)ptr + plan->ws_off[s] : kWsStandIn);
    sp->ws_bound = ptr != nullptr;
    plan->desc[s].b = sp->buf;
    for (int k = 0; k < se::kPasses; ++k) plan->desc[s].pass[k] = sp->passes[k];
  }
  plan->ws_bound = false;
  if (!ptr) return SE_OK;
  // the descriptors the stage kernels read: uploaded once per binding
  if (hipMemcpy(plan->d_sys, plan->desc.data(), sizeof(se::SysDesc) * plan->desc.size(), hipMemcpyHostToDevice) !=
      hipSuccess)
    return SE_ERR_DEVICE;
  plan->ws_bound = true;
  return SE_OK;
}

se_status se_eval_batch(se_batch_plan* plan, const void* xyz, const void* q, void* phi, void* force,
                        double* energy, unsigned flags, void* hip_stream) {
  if (!plan) return SE_ERR_ARG;
  if (!plan->ws_bound) return SE_ERR_WORKSPACE;
  if (plan->total > 0 && (!xyz || !q)) return SE_ERR_ARG;
  if (flags & ~(SE_IN_F32 | SE_ADD_SELF | SE_SYNC_CHECK | SE_OUT_GRAD | SE_ALLOW_NONNEUTRAL | SE_PROFILE))
    return SE_ERR_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  se::BatchIO io{};
  io.xyz = xyz;
  io.q = q;
  io.phi = phi;
  io.force = force;
  io.energy = energy;
  io.in_f32 = (flags & SE_IN_F32) ? 1 : 0;
  io.out_grad = (flags & SE_OUT_GRAD) ? 1 : 0;
  io.add_self = (flags & SE_ADD_SELF) ? 1 : 0;
  io.allow_nonneutral = (flags & SE_ALLOW_NONNEUTRAL) ? 1 : 0;
  io.xcd_tiles = xcd_mode(plan->sys[0]->p.xcd_tiles);
  io.xcd_fft = xcd_mode(plan->sys[0]->p.xcd_fft);
  for (const se_plan* sp : plan->sys)
    for (int k = 0; k < se::kPasses; ++k)
      if (sp->passes[k].wide) io.fft_wide |= 1 << k;
  io.fft_rec = plan->d_rec;
  const bool prof = (flags & SE_PROFILE) != 0;
  if (prof && !plan->have_ev) {
    for (hipEvent_t& e : plan->ev)
      if (hipEventCreate(&e) != hipSuccess) return SE_ERR_DEVICE;
    plan->have_ev = true;
  }
  // the previous profiled evaluation: fold its times in before reusing the events
  if (prof && plan->collect() != SE_OK) return SE_ERR_DEVICE;
  if (se::launch_batch(plan->P, plan->f64, plan->d_sys, (int)plan->sys.size(), plan->d_off, plan->items, io,
                       plan->lds, st, prof ? plan->ev : nullptr) != hipSuccess)
    return SE_ERR_DEVICE;
  if (prof) plan->prof_pending = 1;
  if (flags & SE_SYNC_CHECK) return se_batch_get_device_status(plan, hip_stream);
  return SE_OK;
}

se_status se_batch_plan_profile(se_batch_plan* plan, void* hip_stream, se_stage_record* out, int cap, int* n,
                                int reset) {
  if (!plan || !out || !n || cap < 0) return SE_ERR_ARG;
  if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return SE_ERR_DEVICE;
  if (plan->collect() != SE_OK) return SE_ERR_DEVICE;
  int k_out = 0;
  double ms_all = 0.0, by_all = 0.0, fl_all = 0.0;
  for (int k = 0; k < se::BS_COUNT; ++k) {
    ms_all += plan->st_ms[k];
    by_all += plan->st_bytes[k];
    fl_all += plan->st_flops[k];
    if (plan->items[k] == 0 || k_out >= cap) continue;
    se_stage_record& r = out[k_out++];
    std::memset(&r, 0, sizeof(r));
    std::snprintf(r.name, sizeof(r.name), "%s", kBatchStageNames[k]);
    r.launches = plan->prof_launches;
    r.ms_total = plan->st_ms[k];
    r.bytes = plan->st_bytes[k];
    r.flops = plan->st_flops[k];
  }
  if (k_out < cap) {
    se_stage_record& r = out[k_out++];
    std::memset(&r, 0, sizeof(r));
    std::snprintf(r.name, sizeof(r.name), "batch_all_stages");
    r.launches = plan->prof_launches;
    r.ms_total = ms_all;
    r.bytes = by_all;
    r.flops = fl_all;
  }
  *n = k_out;
  if (reset) {
    for (double& m : plan->st_ms) m = 0.0;
    plan->prof_launches = 0;
  }
  return SE_OK;
}

se_status se_batch_get_device_status(se_batch_plan* plan, void* hip_stream) {
  if (!plan) return SE_ERR_ARG;
  se_status worst = SE_OK;
  for (se_plan* s : plan->sys) {
    const se_status r = se_get_device_status(s, hip_stream);
    if (r == SE_ERR_NONFINITE || (r != SE_OK && worst == SE_OK) ||
        (r == SE_ERR_OUT_OF_BOX && worst == SE_ERR_NONNEUTRAL))
      worst = r;
  }
  return worst;
}

se_status se_batch_plan_destroy(se_batch_plan* plan) {
  if (plan) {
    (void)hipSetDevice(plan->device);
    delete plan;
  }
  return SE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner: picks the schedule knobs of a plan (tile shape, FFT samples per
// workgroup, XCD mapping) by timing candidates on the caller's own input with
// the plans' HIP event profiles.  Tile knobs only change the spread, fold and
// gather launches and FFT knobs only the transform passes, so the two groups
// are tuned one after the other against the times of their own launches.
// ---------------------------------------------------------------------------
namespace {

struct TuneTimes {
  double tiles = 0.0, fft = 0.0, all = 0.0;
};

void classify(const se_stage_record* r, int n, TuneTimes* t) {
  for (int i = 0; i < n; ++i) {
    if (!std::strcmp(r[i].name, "batch_all_stages") || r[i].launches == 0) continue;
    const double ms = r[i].ms_total / r[i].launches;
    t->all += ms;
    if (!std::strcmp(r[i].name, "spread") || !std::strcmp(r[i].name, "fold") || !std::strcmp(r[i].name, "gather") ||
        !std::strcmp(r[i].name, "order") || !std::strcmp(r[i].name, "scatter"))
      t->tiles += ms;
    else if (!std::strncmp(r[i].name, "fft", 3))
      t->fft += ms;
  }
}

constexpr int kTuneWarm = 2, kTuneReps = 5;
const int kTuneTiles[][3] = {{16, 16, 16}, {32, 16, 8}, {32, 8, 8}, {16, 16, 8},
                             {16, 8, 8},   {8, 8, 8},   {8, 8, 4},  {4, 4, 4}};
const int kTuneCaps[] = {1024, 2048, 4096, 8192};
const int kTuneXcd[] = {-1, 8, 32};   // plain order, chunks of 8, chunks of 32 (besides the default)

struct TuneIO {
  const void* xyz;
  const void* q;
  void* phi;
  void* force;
  double* energy;
  unsigned flags;
  void* st;
};

// Device memory the tuner allocates for its own runs (outputs, workspaces).
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bool alloc(size_t n) { return hipMalloc(&p, std::max<size_t>(n, 16)) == hipSuccess; }
};

// One candidate for a single system; false if it cannot be planned or run.
bool time_single(const se_params& p, long N, const TuneIO& io, TuneTimes* t) {
  se_plan* pl = nullptr;
  if (se_plan_create(&p, N, io.st, &pl) != SE_OK) return false;
  DevBuf ws;
  size_t wb = 0;
  if (se_plan_workspace_size(pl, &wb) != SE_OK || !ws.alloc(wb) || se_plan_set_workspace(pl, ws.p, wb) != SE_OK) {
    se_plan_destroy(pl);
    return false;
  }
  se_stage_record rec[32];
  int n = 0;
  bool ok = true;
  for (int i = 0; i < kTuneWarm && ok; ++i)
    ok = se_eval(pl, N, io.xyz, io.q, io.phi, io.force, io.energy, io.flags, io.st) == SE_OK;
  ok = ok && se_plan_profile(pl, io.st, rec, 32, &n, 1) == SE_OK;
  for (int i = 0; i < kTuneReps && ok; ++i)
    ok = se_eval(pl, N, io.xyz, io.q, io.phi, io.force, io.energy, io.flags | SE_PROFILE, io.st) == SE_OK;
  ok = ok && se_plan_profile(pl, io.st, rec, 32, &n, 1) == SE_OK;
  if (ok) classify(rec, n, t);
  se_plan_destroy(pl);
  return ok;
}

bool time_batch(const std::vector<se_params>& p, const std::vector<long>& N, const TuneIO& io, TuneTimes* t) {
  se_batch_plan* bp = nullptr;
  if (se_batch_plan_create(p.data(), N.data(), (int)p.size(), io.st, &bp) != SE_OK) return false;
  DevBuf ws;
  size_t wb = 0;
  if (se_batch_plan_workspace_size(bp, &wb) != SE_OK || !ws.alloc(wb) ||
      se_batch_plan_set_workspace(bp, ws.p, wb) != SE_OK) {
    se_batch_plan_destroy(bp);
    return false;
  }
  se_stage_record rec[32];
  int n = 0;
  bool ok = true;
  for (int i = 0; i < kTuneWarm && ok; ++i)
    ok = se_eval_batch(bp, io.xyz, io.q, io.phi, io.force, io.energy, io.flags, io.st) == SE_OK;
  ok = ok && se_batch_plan_profile(bp, io.st, rec, 32, &n, 1) == SE_OK;
  for (int i = 0; i < kTuneReps && ok; ++i)
    ok = se_eval_batch(bp, io.xyz, io.q, io.phi, io.force, io.energy, io.flags | SE_PROFILE, io.st) == SE_OK;
  ok = ok && se_batch_plan_profile(bp, io.st, rec, 32, &n, 1) == SE_OK;
  if (ok) classify(rec, n, t);
  se_batch_plan_destroy(bp);
  return ok;
}

// Coordinate search over the knob groups.  timer(params, times) times one
// setting; set(params, knob...) edits a copy.  Returns false if not even the
// default setting runs.
template <typename Timer>
bool tune_knobs(se_params* base, int n_par, bool tune_xcd, Timer timer, se_tune_report* rep) {
  auto with = [&](auto edit) {
    std::vector<se_params> v(base, base + n_par);
    for (auto& p : v) edit(p);
    return v;
  };
  TuneTimes t0;
  std::vector<se_params> cur(base, base + n_par);
  if (!timer(cur, &t0)) return false;
  int cand = 1;
  // spreading mode and tile shape (with the current XCD setting)
  double best = t0.tiles;
  for (int mode : {1, 2, 3})
    for (const auto& T : kTuneTiles) {
      auto v = with([&](se_params& p) {
        p.tile = 0;
        p.spread_mode = mode;
        for (int d = 0; d < 3; ++d) p.tile3[d] = T[d];
      });
      TuneTimes t;
      if (!timer(v, &t)) continue;
      ++cand;
      if (t.tiles < best) {
        best = t.tiles;
        cur = v;
      }
    }
  if (tune_xcd) {
    const auto base_v = cur;
    for (int mode : kTuneXcd) {
      auto v = base_v;
      for (auto& p : v) p.xcd_tiles = mode;
      TuneTimes t;
      if (!timer(v, &t)) continue;
      ++cand;
      if (t.tiles < best) {
        best = t.tiles;
        cur = v;
      }
    }
  }
  // FFT samples per workgroup
  TuneTimes tc;
  if (!timer(cur, &tc)) return false;
  best = tc.fft;
  for (int cap : kTuneCaps) {
    auto v = cur;
    for (auto& p : v) p.fft_cap = cap;
    TuneTimes t;
    if (!timer(v, &t)) continue;
    ++cand;
    if (t.fft < best) {
      best = t.fft;
      cur = v;
    }
  }
  if (tune_xcd) {
    const auto base_v = cur;
    for (int mode : kTuneXcd) {
      auto v = base_v;
      for (auto& p : v) p.xcd_fft = mode;
      TuneTimes t;
      if (!timer(v, &t)) continue;
      ++cand;
      if (t.fft < best) {
        best = t.fft;
        cur = v;
      }
    }
  }
  TuneTimes tf;
  if (!timer(cur, &tf)) return false;
  // keep the default if the tuned setting is not faster as a whole
  if (tf.all > t0.all) {
    cur.assign(base, base + n_par);
    tf = t0;
  }
  for (int i = 0; i < n_par; ++i) base[i] = cur[i];
  if (rep) {
    rep->candidates += cand;
    rep->ms_default += t0.all;
    rep->ms_tuned += tf.all;
  }
  return true;
}

}  // namespace

extern "C" {

se_status se_autotune(const se_params* params, long N, const void* xyz, const void* q, unsigned flags,
                      void* hip_stream, se_params* tuned, se_tune_report* report) {
  if (!params || !tuned || N < 1 || !xyz || !q) return SE_ERR_ARG;
  if (flags & ~(SE_IN_F32 | SE_ALLOW_NONNEUTRAL)) return SE_ERR_ARG;
  if (report) std::memset(report, 0, sizeof(*report));
  const size_t re = params->prec == SE_F64 ? 8 : 4;
  DevBuf phi, force, energy;
  if (!phi.alloc(re * N) || !force.alloc(3 * re * N) || !energy.alloc(8)) return SE_ERR_NOMEM;
  TuneIO io{xyz, q, phi.p, force.p, (double*)energy.p, flags, hip_stream};
  se_params p = *params;
  auto timer = [&](const std::vector<se_params>& v, TuneTimes* t) { return time_single(v[0], N, io, t); };
  if (!tune_knobs(&p, 1, true, timer, report)) return SE_ERR_UNSUPPORTED;
  *tuned = p;
  return SE_OK;
}

se_status se_batch_autotune(const se_params* params, const long* N, int n_sys, const void* xyz, const void* q,
                            unsigned flags, void* hip_stream, se_params* tuned, se_tune_report* report) {
  if (!params || !N || !tuned || n_sys < 1 || !xyz || !q) return SE_ERR_ARG;
  if (flags & ~(SE_IN_F32 | SE_ALLOW_NONNEUTRAL)) return SE_ERR_ARG;
  if (report) std::memset(report, 0, sizeof(*report));
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<long> off(n_sys + 1, 0);
  for (int s = 0; s < n_sys; ++s) {
    if (N[s] < 0) return SE_ERR_ARG;
    off[s + 1] = off[s] + N[s];
  }
  const long total = off[n_sys];
  const size_t re = params[0].prec == SE_F64 ? 8 : 4, ie = (flags & SE_IN_F32) ? 4 : 8;
  DevBuf phi, force, energy, gx, gq;
  if (!phi.alloc(re * total) || !force.alloc(3 * re * total) || !energy.alloc(8 * n_sys) ||
      !gx.alloc(3 * ie * total) || !gq.alloc(ie * total))
    return SE_ERR_NOMEM;
  std::vector<se_params> out(params, params + n_sys);
  // tile and FFT knobs per periodicity class, on that class's systems alone
  for (int D = 0; D <= 3; ++D) {
    std::vector<int> idx;
    for (int s = 0; s < n_sys; ++s)
      if (params[s].D == D) idx.push_back(s);
    if (idx.empty()) continue;
    std::vector<se_params> sub;
    std::vector<long> subN;
    long run = 0;
    for (int s : idx) {
      sub.push_back(params[s]);
      subN.push_back(N[s]);
      if (N[s] > 0 &&
          (hipMemcpyAsync((char*)gx.p + 3 * ie * run, (const char*)xyz + 3 * ie * off[s], 3 * ie * N[s],
                          hipMemcpyDeviceToDevice, st) != hipSuccess ||
           hipMemcpyAsync((char*)gq.p + ie * run, (const char*)q + ie * off[s], ie * N[s],
                          hipMemcpyDeviceToDevice, st) != hipSuccess))
        return SE_ERR_DEVICE;
      run += N[s];
    }
    TuneIO io{gx.p, gq.p, phi.p, force.p, (double*)energy.p, flags, hip_stream};
    auto timer = [&](const std::vector<se_params>& v, TuneTimes* t) { return time_batch(v, subN, io, t); };
    se_tune_report r{};
    if (!tune_knobs(sub.data(), (int)sub.size(), false, timer, &r)) return SE_ERR_UNSUPPORTED;
    if (report) report->candidates += r.candidates;
    for (size_t k = 0; k < idx.size(); ++k) out[idx[k]] = sub[k];
  }
  // XCD mapping (one setting for the whole batch) on the full batch
  {
    TuneIO io{xyz, q, phi.p, force.p, (double*)energy.p, flags, hip_stream};
    std::vector<long> vN(N, N + n_sys);
    TuneTimes t0, tb;
    std::vector<se_params> def(params, params + n_sys);
    if (!time_batch(def, vN, io, &t0)) return SE_ERR_UNSUPPORTED;
    if (!time_batch(out, vN, io, &tb)) return SE_ERR_UNSUPPORTED;
    int cand = 2;
    // One transform launch takes the largest LDS of all its systems, so the
    // samples cap chosen per class is checked against each chosen value used
    // for every system, on the whole batch.
    std::vector<int> caps;
    for (const auto& p : out)
      if (std::find(caps.begin(), caps.end(), p.fft_cap) == caps.end()) caps.push_back(p.fft_cap);
    if (caps.size() > 1)
      for (int cap : caps) {
        auto v = out;
        for (auto& p : v) p.fft_cap = cap;
        TuneTimes t;
        if (!time_batch(v, vN, io, &t)) continue;
        ++cand;
        if (t.fft < tb.fft) {
          tb = t;
          out = v;
        }
      }
    for (int group = 0; group < 2; ++group) {
      const auto base_v = out;
      for (int mode : kTuneXcd) {
        auto v = base_v;
        for (auto& p : v) (group == 0 ? p.xcd_tiles : p.xcd_fft) = mode;
        TuneTimes t;
        if (!time_batch(v, vN, io, &t)) continue;
        ++cand;
        if ((group == 0 ? t.tiles < tb.tiles : t.fft < tb.fft)) {
          tb = t;
          out = v;
        }
      }
    }
    if (tb.all > t0.all) {
      out = def;
      tb = t0;
    }
    if (report) {
      report->candidates += cand;
      report->ms_default = t0.all;
      report->ms_tuned = tb.all;
    }
  }
  for (int s = 0; s < n_sys; ++s) tuned[s] = out[s];
  return SE_OK;
}

}  // extern "C"
