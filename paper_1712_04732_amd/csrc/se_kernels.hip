// gfx950 kernels of the Spectral Ewald k-space path (Algorithm 4 of
// Shamshirgar, Bagge, Tornberg, arXiv:1712.04732).
//
//   bin      : grid cell, fractional offset and tile of every particle; tile
//              counting sort (implementation of the gridding loop bounds).
//   spread   : Eq. (gridding).  Output-stationary: one workgroup owns one tile
//              of the grid, accumulates every particle whose P^3 stencil meets
//              the tile into an LDS copy of the tile, and writes the tile once.
//              No global atomics; grid bytes are written exactly once.
//   fft      : mixed-radix (2,3,4,5,7,8) Stockham pencil transforms in LDS,
//              with zero padding on load and truncation on store (the padded
//              free-direction transforms of Algorithm 1/2 and the (2 Mt)^3
//              free-space transform), and a fused variant that runs forward
//              transform, scaling by Eq. (scale) and inverse transform on a
//              pencil without leaving LDS.
//   gather   : trapezoidal rule of Eq. (complete_integral) and its gradient,
//              Eq. (force-method-1).  One workgroup per tile stages the
//              tile's stencil region of the grid in LDS; one wavefront per
//              particle, 64 lanes over the stencil columns, cross-lane
//              reduction by shuffles.
//   energy   : FP64 reduction of q phi.
//   0P       : Algorithm 3 helpers in FP64.
#include <hip/hip_runtime.h>

#include "se_internal.h"

namespace se {

template <typename T>
struct __align__(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return {a.re * s, a.im * s};
}
// multiply by sign * i
template <typename T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a, int sign) {
  return sign > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

template <typename T>
struct Quad {
  T fx, fy, fz, q;
};

// ---------------------------------------------------------------------------
// Small DFTs, X_m = sum_r v_r exp(sign 2 pi i r m / R)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  const cx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>* v, int sign) {
  const cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3];
  const cx<T> t3 = mul_si(v[1] - v[3], sign);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <typename T>
__device__ __forceinline__ void dft8(cx<T>* v, int sign) {
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e, sign);
  dft4(o, sign);
  const T c = (T)0.70710678118654752440;
  // w^k = exp(sign i pi k / 4)
  const cx<T> o1 = cmul(o[1], cx<T>{c, sign * c});
  const cx<T> o2 = mul_si(o[2], sign);
  const cx<T> o3 = cmul(o[3], cx<T>{-c, sign * c});
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

// Odd radix R in {3,5,7}: pair r with R-r,
//   X_m = v_0 + sum_{r=1}^{(R-1)/2} [(v_r + v_{R-r}) cos(2 pi r m/R)
//                                  + sign i (v_r - v_{R-r}) sin(2 pi r m/R)].
template <int R>
struct OddRoots;
template <>
struct OddRoots<3> {
  static constexpr double c[3] = {1.0, -0.5, -0.5};
  static constexpr double s[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
};
template <>
struct OddRoots<5> {
  static constexpr double c[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410,
                                  -0.80901699437494742410, 0.30901699437494742410};
  static constexpr double s[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917,
                                  -0.58778525229247312917, -0.95105651629515357212};
};
template <>
struct OddRoots<7> {
  static constexpr double c[7] = {1.0,
                                  0.62348980185873353053,
                                  -0.22252093395631440429,
                                  -0.90096886790241912624,
                                  -0.90096886790241912624,
                                  -0.22252093395631440429,
                                  0.62348980185873353053};
  static constexpr double s[7] = {0.0,
                                  0.78183148246802980871,
                                  0.97492791218182360702,
                                  0.43388373911755812048,
                                  -0.43388373911755812048,
                                  -0.97492791218182360702,
                                  -0.78183148246802980871};
};

template <typename T, int R>
__device__ __forceinline__ void dft_odd(cx<T>* v, int sign) {
  constexpr int H = (R - 1) / 2;
  cx<T> a[H], b[H];
  cx<T> x0 = v[0];
#pragma unroll
  for (int r = 1; r <= H; ++r) {
    a[r - 1] = v[r] + v[R - r];
    b[r - 1] = v[r] - v[R - r];
    x0 = x0 + a[r - 1];
  }
  cx<T> out[R];
  out[0] = x0;
#pragma unroll
  for (int m = 1; m < R; ++m) {
    cx<T> acc = v[0];
    cx<T> bs = {0, 0};
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      const int j = (r * m) % R;
      const T cc = (T)OddRoots<R>::c[j], ss = (T)OddRoots<R>::s[j];
      acc = acc + cscale(a[r - 1], cc);
      bs = bs + cscale(b[r - 1], ss);
    }
    out[m] = acc + mul_si(bs, sign);
  }
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = out[m];
}

template <typename T, int R>
__device__ __forceinline__ void dft(cx<T>* v, int sign) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 4) dft4(v, sign);
  else if constexpr (R == 8) dft8(v, sign);
  else dft_odd<T, R>(v, sign);
}

// One Stockham stage over B interleaved pencils (sample-major, index t*B + p):
//   input  j + r n/R   (j = 0..n/R-1)
//   twiddle exp(sign 2 pi i r k/(Ns R)), k = j mod Ns
//   output (j/Ns) Ns R + k + r Ns
template <typename T, int R>
__device__ __forceinline__ void fft_stage(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                          const cx<T>* __restrict__ tw, int n, int Ns, int B,
                                          int sign) {
  const int nb = n / R;
  const int total = nb * B;
  const int tws = n / (Ns * R);
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int j = e / B, p = e - (e / B) * B;
    const int k = j % Ns;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(j + r * nb) * B + p];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = tw[r * k * tws];  // r k tws < R Ns tws = n
        if (sign > 0) w.im = -w.im;
        v[r] = cmul(v[r], w);
      }
    }
    dft<T, R>(v, sign);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(base + r * Ns) * B + p] = v[r];
  }
}

// Runs all stages of class C; returns the buffer holding the result.
template <typename T>
__device__ cx<T>* fft_run(cx<T>* b0, cx<T>* b1, const cx<T>* tw, const FftClass& C, int B,
                          int sign) {
  cx<T>* src = b0;
  cx<T>* dst = b1;
  int Ns = 1;
  for (int s = 0; s < C.nst; ++s) {
    const int R = C.rad[s];
    switch (R) {
      case 2: fft_stage<T, 2>(src, dst, tw, C.n, Ns, B, sign); break;
      case 3: fft_stage<T, 3>(src, dst, tw, C.n, Ns, B, sign); break;
      case 4: fft_stage<T, 4>(src, dst, tw, C.n, Ns, B, sign); break;
      case 5: fft_stage<T, 5>(src, dst, tw, C.n, Ns, B, sign); break;
      case 7: fft_stage<T, 7>(src, dst, tw, C.n, Ns, B, sign); break;
      default: fft_stage<T, 8>(src, dst, tw, C.n, Ns, B, sign); break;
    }
    __syncthreads();
    cx<T>* tmp = src;
    src = dst;
    dst = tmp;
    Ns *= R;
  }
  return src;
}

__device__ __forceinline__ int fold_index(int i, int n) { return i <= n - i ? i : n - i; }

template <typename T>
__device__ __forceinline__ T scale_factor(const FftClass& C, int b0, int b1, int t) {
  const T* sA = (const T*)C.sA;
  const T* sB = (const T*)C.sB;
  const T* sC = (const T*)C.sC;
  T s = sA[b0 + C.offA] * sB[b1 + C.offB] * sC[t];
  const T* gt = (const T*)C.gtab;
  switch (C.gmode) {
    case G_INVSQ: {
      const T k2 = ((const T*)C.kA)[b0 + C.offA] + ((const T*)C.kB)[b1 + C.offB] + ((const T*)C.kC)[t];
      return k2 > (T)0 ? s / k2 : (T)0;
    }
    case G_TAB1:
      return s * gt[t];
    case G_TAB2: {
      const int i0 = C.fold0 ? fold_index(b0, C.fold0) : b0;
      return s * gt[(long long)i0 * C.gd2 + fold_index(t, C.fold2)];
    }
    case G_TAB3: {
      const int i0 = C.fold0 ? fold_index(b0, C.fold0) : b0;
      return s * gt[((long long)i0 * C.gd1 + fold_index(b1, C.fold1)) * C.gd2 + fold_index(t, C.fold2)];
    }
    default:
      return s;
  }
}

template <typename T, int KIND>
__global__ __launch_bounds__(kBlock) void fft_kernel(const FftPass P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 it = P.items[blockIdx.x];
  const FftClass& C = P.cls[it.x];
  const int n = C.n, B = P.B, cnt = it.w, b0s = it.y, b1 = it.z;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem);
  cx<T>* buf0 = tw + P.nmax;
  cx<T>* buf1 = buf0 + (size_t)B * P.nmax;

  const cx<T>* twg = reinterpret_cast<const cx<T>*>(C.tw);
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = twg[i];

  // ---- load B pencils, zero padded to n ----
  const bool t_fast = (C.in_st == 1);
  const int total = n * B;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int t, p;
    if (t_fast) {
      p = e / n;
      t = e - p * n;
    } else {
      t = e / B;
      p = e - t * B;
    }
    cx<T> v = {0, 0};
    if (p < cnt) {
      const long long base = (long long)(b0s + p) * C.in_s0 + (long long)b1 * C.in_s1;
      if constexpr (KIND == K_R2C) {
        if (t < C.n_in) v.re = reinterpret_cast<const T*>(C.in)[base + (long long)t * C.in_st];
      } else if constexpr (KIND == K_C2R) {
        // Hermitian extension of the stored half spectrum (t <= n/2)
        const int h = n >> 1;
        const int ts = t <= h ? t : n - t;
        v = reinterpret_cast<const cx<T>*>(C.in)[base + (long long)ts * C.in_st];
        if (t > h) v.im = -v.im;
      } else {
        if (t < C.n_in) v = reinterpret_cast<const cx<T>*>(C.in)[base + (long long)t * C.in_st];
      }
    }
    buf0[t * B + p] = v;
  }
  __syncthreads();

  cx<T>* res;
  if constexpr (KIND == K_C2C_INV || KIND == K_C2R) {
    res = fft_run<T>(buf0, buf1, tw, C, B, +1);
  } else {
    res = fft_run<T>(buf0, buf1, tw, C, B, -1);
  }

  if constexpr (KIND == K_FUSED) {
    // scaling step, Eq. (scale), on the spectrum of each pencil
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int t = e / B, p = e - (e / B) * B;
      if (p < cnt) res[e] = cscale(res[e], scale_factor<T>(C, b0s + p, b1, t));
    }
    __syncthreads();
    cx<T>* other = (res == buf0) ? buf1 : buf0;
    res = fft_run<T>(res, other, tw, C, B, +1);
  }

  // ---- store the first n_out samples ----
  const bool to_fast = (C.out_st == 1);
  const int totout = C.n_out * B;
  for (int e = threadIdx.x; e < totout; e += blockDim.x) {
    int t, p;
    if (to_fast) {
      p = e / C.n_out;
      t = e - p * C.n_out;
    } else {
      t = e / B;
      p = e - t * B;
    }
    if (p >= cnt) continue;
    const long long base = (long long)(b0s + p) * C.out_s0 + (long long)b1 * C.out_s1;
    const cx<T> v = res[t * B + p];
    if constexpr (KIND == K_C2R) {
      reinterpret_cast<T*>(C.out)[base + (long long)t * C.out_st] = v.re;
    } else {
      reinterpret_cast<cx<T>*>(C.out)[base + (long long)t * C.out_st] = v;
    }
  }
}

size_t fft_lds_bytes(const FftPass& p, bool f64) {
  const size_t c = f64 ? 16 : 8;
  return c * ((size_t)p.nmax + 2 * (size_t)p.B * p.nmax);
}

template <typename T>
static hipError_t launch_fft_t(const FftPass& p, hipStream_t st) {
  if (p.nitems <= 0) return hipSuccess;
  const size_t lds = fft_lds_bytes(p, sizeof(T) == 8);
  const dim3 grid(p.nitems), block(kBlock);
  switch (p.kind) {
    case K_C2C_FWD: fft_kernel<T, K_C2C_FWD><<<grid, block, lds, st>>>(p); break;
    case K_C2C_INV: fft_kernel<T, K_C2C_INV><<<grid, block, lds, st>>>(p); break;
    case K_R2C: fft_kernel<T, K_R2C><<<grid, block, lds, st>>>(p); break;
    case K_C2R: fft_kernel<T, K_C2R><<<grid, block, lds, st>>>(p); break;
    default: fft_kernel<T, K_FUSED><<<grid, block, lds, st>>>(p); break;
  }
  return hipGetLastError();
}

hipError_t launch_fft(const FftPass& p, bool f64, hipStream_t st) {
  return f64 ? launch_fft_t<double>(p, st) : launch_fft_t<float>(p, st);
}

// ---------------------------------------------------------------------------
// Binning
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pack_cell(int cx_, int cy, int cz) { return cx_ | (cy << 10) | (cz << 20); }

template <typename T>
__device__ __forceinline__ T warp_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <typename Tin, typename T>
__global__ __launch_bounds__(kBlock) void bin_kernel(GridGeom g, EvalBuffers b, long N,
                                                     const Tin* __restrict__ xyz,
                                                     const Tin* __restrict__ q) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0, sa = 0.0, s2 = 0.0;
  if (n < N) {
    double qn = (double)q[n];
    int c[3];
    double f[3];
    int bad = 0;
    if (!isfinite(qn)) bad |= 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = (double)xyz[3 * n + d];
      int ci;
      double t;
      if (!isfinite(x)) {
        bad |= 1;
        ci = g.per[d] ? 0 : g.d0[d];
        t = (double)ci;
      } else if (g.per[d]) {
        const double xw = x - g.L * floor(x / g.L);
        t = xw / g.h;
        ci = (int)floor(t);
        if (ci >= g.G[d]) {  // xw rounded up to L
          ci = 0;
          t = 0.0;
        }
        if (ci < 0) {
          ci = 0;
          t = 0.0;
        }
      } else {
        if (!(x >= 0.0 && x < g.L)) bad |= 2;
        t = x / g.h + g.d0[d];
        ci = (int)floor(t);
        const int lo = g.d0[d], hi = g.d0[d] + (g.G[d] - 2 * g.d0[d]) - 1;
        if (ci < lo) {
          ci = lo;
          t = (double)lo;
        }
        if (ci > hi) {
          ci = hi;
          t = fmin(t, (double)hi + 1.0);
        }
      }
      c[d] = ci;
      f[d] = t - (double)ci;
    }
    if (bad) {
      atomicOr(b.status, bad);
      qn = 0.0;
    }
    const int tile = ((c[2] / g.tile) * g.nt[1] + c[1] / g.tile) * g.nt[0] + c[0] / g.tile;
    b.p_tile[n] = tile;
    b.p_cell[n] = pack_cell(c[0], c[1], c[2]);
    reinterpret_cast<Quad<T>*>(b.p_frac)[n] = Quad<T>{(T)f[0], (T)f[1], (T)f[2], (T)qn};
    atomicAdd(&b.tile_count[tile], 1);
    sq = qn;
    sa = fabs(qn);
    s2 = qn * qn;
  }
  // block partial sums of the charges (FP64), for the neutrality check and Q
  __shared__ double red[3][kBlock / 64];
  sq = warp_sum(sq);
  sa = warp_sum(sa);
  s2 = warp_sum(s2);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) {
    red[0][w] = sq;
    red[1][w] = sa;
    red[2][w] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) s += red[threadIdx.x][i];
    b.qpart[3 * blockIdx.x + threadIdx.x] = s;
  }
}

hipError_t launch_bin(const GridGeom& g, const EvalBuffers& b, long N, const void* xyz,
                      const void* q, bool in_f32, bool f64, int nblk, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  const dim3 grid(nblk), block(kBlock);
  if (in_f32) {
    if (f64)
      bin_kernel<float, double><<<grid, block, 0, st>>>(g, b, N, (const float*)xyz, (const float*)q);
    else
      bin_kernel<float, float><<<grid, block, 0, st>>>(g, b, N, (const float*)xyz, (const float*)q);
  } else {
    if (f64)
      bin_kernel<double, double><<<grid, block, 0, st>>>(g, b, N, (const double*)xyz, (const double*)q);
    else
      bin_kernel<double, float><<<grid, block, 0, st>>>(g, b, N, (const double*)xyz, (const double*)q);
  }
  return hipGetLastError();
}

// Exclusive scan of the tile counts (one workgroup of 1024 threads), the
// cursors of the scatter, and the FP64 charge sums with the neutrality check.
__global__ __launch_bounds__(1024) void scan_kernel(GridGeom g, EvalBuffers b, int nblk_bin,
                                                    int check_neutral) {
  const int ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  const int T = blockDim.x;
  const int per = (ntiles + T - 1) / T;
  const int lo = threadIdx.x * per;
  const int hi = min(ntiles, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += b.tile_count[i];
  __shared__ int part[1024];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int i = lo; i < hi; ++i) {
    b.tile_start[i] = run;
    b.tile_cursor[i] = run;
    run += b.tile_count[i];
  }
  if (threadIdx.x == T - 1) b.tile_start[ntiles] = part[T - 1];

  __shared__ double dq[3][1024];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < nblk_bin; i += T) {
    a0 += b.qpart[3 * i];
    a1 += b.qpart[3 * i + 1];
    a2 += b.qpart[3 * i + 2];
  }
  dq[0][threadIdx.x] = a0;
  dq[1][threadIdx.x] = a1;
  dq[2][threadIdx.x] = a2;
  __syncthreads();
  if (threadIdx.x < 3) {
    double acc = 0.0;
    for (int i = 0; i < T; ++i) acc += dq[threadIdx.x][i];
    b.red[threadIdx.x] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0 && check_neutral) {
    const double Q = b.red[0], A = b.red[1];
    if (fabs(Q) > 1e-10 * A) atomicOr(b.status, 4);
  }
}

hipError_t launch_scan(const GridGeom& g, const EvalBuffers& b, int nblk_bin, int check_neutral,
                       hipStream_t st) {
  scan_kernel<<<dim3(1), dim3(1024), 0, st>>>(g, b, nblk_bin, check_neutral);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scatter_kernel(EvalBuffers b, long N) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int tile = b.p_tile[n];
  const int pos = atomicAdd(&b.tile_cursor[tile], 1);
  b.s_cell[pos] = b.p_cell[n];
  b.s_idx[pos] = (int)n;
  reinterpret_cast<Quad<T>*>(b.s_fq)[pos] = reinterpret_cast<const Quad<T>*>(b.p_frac)[n];
}

hipError_t launch_scatter(const GridGeom& g, const EvalBuffers& b, long N, bool f64, hipStream_t st) {
  (void)g;
  if (N <= 0) return hipSuccess;
  const dim3 grid((unsigned)((N + kBlock - 1) / kBlock)), block(kBlock);
  if (f64)
    scatter_kernel<double><<<grid, block, 0, st>>>(b, N);
  else
    scatter_kernel<float><<<grid, block, 0, st>>>(b, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window weights (Section 4).  f = frac(t) of the particle's grid coordinate,
// stencil point i at grid index floor(t) - P/2 + 1 + i.
//   PKB: xbar = 1 - 2f for all i (Section 4.1), Horner per subinterval;
//        derivative table already holds d/dx (chain factor -2/h).
//   Gaussian: u = i + 1 - P/2 - f (grid units), W = exp(-alpha (2u/P)^2),
//        dW/dx = W 2 alpha (2/P)^2 u / h.
// ---------------------------------------------------------------------------
template <typename T, int P>
__device__ __forceinline__ void window_weights(const GridGeom& g, const T* __restrict__ coef,
                                               const T* __restrict__ dcoef, T f, T* w, T* dw) {
  if (g.window == 1) {
    const T xb = (T)1 - (T)2 * f;
    const int m = g.nu + 1;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      T a = coef[i * m + g.nu];
      for (int j = g.nu - 1; j >= 0; --j) a = a * xb + coef[i * m + j];
      w[i] = a;
      if (dw) {
        T d = dcoef[i * m + g.nu];
        for (int j = g.nu - 1; j >= 0; --j) d = d * xb + dcoef[i * m + j];
        dw[i] = d;
      }
    }
  } else {
    const T a = (T)g.alpha;
    const T c2 = (T)4 / (T)(P * P);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const T u = (T)(i + 1 - P / 2) - f;
      const T e = exp(-a * c2 * u * u);
      w[i] = e;
      if (dw) dw[i] = e * (T)2 * a * c2 * u / (T)g.h;
    }
  }
}

// Tiles of one direction that hold anchor cells of particles whose stencil
// meets the tile [x0, x0 + ext).  Anchor cells c with c - P/2 + 1 <= x0 + ext - 1
// and c + P/2 >= x0, wrapped in periodic directions.
__device__ __forceinline__ int neighbor_tiles(int x0, int ext, int G, int per, int tile, int P,
                                              int* list) {
  int cnt = 0;
  const int lo = x0 - P / 2, hi = x0 + ext - 2 + P / 2;
  for (int c = lo; c <= hi; ++c) {
    int cc = c;
    if (per) {
      cc = c % G;
      if (cc < 0) cc += G;
    } else if (c < 0 || c >= G) {
      continue;
    }
    const int t = cc / tile;
    bool seen = false;
    for (int k = 0; k < cnt; ++k) seen |= (list[k] == t);
    if (!seen && cnt < 8) list[cnt++] = t;
  }
  return cnt;
}


template <typename T, int P>
__global__ __launch_bounds__(kBlock) void spread_kernel(GridGeom g, EvalBuffers b) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TT = g.tile;
  const int tz = blockIdx.x / (g.nt[0] * g.nt[1]);
  const int ty = (blockIdx.x / g.nt[0]) % g.nt[1];
  const int tx = blockIdx.x % g.nt[0];
  const int x0 = tx * TT, y0 = ty * TT, z0 = tz * TT;
  const int ex = min(TT, g.G[0] - x0), ey = min(TT, g.G[1] - y0), ez = min(TT, g.G[2] - z0);
  const int m = g.nu + 1;

  const int kChunk = g.chunk;
  T* acc = reinterpret_cast<T*>(smem);                  // TT^3
  T* wx = acc + TT * TT * TT;                            // kChunk * P
  T* wy = wx + kChunk * P;
  T* wz = wy + kChunk * P;
  T* coef = wz + kChunk * P;                             // P * m
  int* off = reinterpret_cast<int*>(coef + P * m);       // kChunk * 3
  int* ncomp = off + 3 * kChunk;

  for (int i = threadIdx.x; i < TT * TT * TT; i += blockDim.x) acc[i] = (T)0;
  for (int i = threadIdx.x; i < P * m; i += blockDim.x) coef[i] = reinterpret_cast<const T*>(b.wtab)[i];
  if (threadIdx.x == 0) *ncomp = 0;

  int lx[8], ly[8], lz[8];
  const int nx = neighbor_tiles(x0, ex, g.G[0], g.per[0], TT, P, lx);
  const int ny = neighbor_tiles(y0, ey, g.G[1], g.per[1], TT, P, ly);
  const int nz = neighbor_tiles(z0, ez, g.G[2], g.per[2], TT, P, lz);
  __syncthreads();

  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwaves = blockDim.x / 64;
  const Quad<T>* sfq = reinterpret_cast<const Quad<T>*>(b.s_fq);

  for (int a = 0; a < nz; ++a)
    for (int bb = 0; bb < ny; ++bb)
      for (int c = 0; c < nx; ++c) {
        const int nt = (lz[a] * g.nt[1] + ly[bb]) * g.nt[0] + lx[c];
        const int start = b.tile_start[nt], end = b.tile_start[nt + 1];
        for (int base = start; base < end; base += kChunk) {
          // 1. select particles whose stencil meets this tile; window weights
          const int i = base + threadIdx.x;
          if (threadIdx.x < kChunk && i < end) {
            const int pc = b.s_cell[i];
            const int cc[3] = {pc & 1023, (pc >> 10) & 1023, (pc >> 20) & 1023};
            const int org[3] = {x0, y0, z0}, ext[3] = {ex, ey, ez};
            int o[3];
            bool hit = true;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              int od = cc[d] - P / 2 + 1 - org[d];
              if (g.per[d]) {
                od %= g.G[d];
                if (od < 0) od += g.G[d];
                hit = hit && (od < ext[d] || od + P > g.G[d]);
              } else {
                hit = hit && (od < ext[d] && od + P > 0);
              }
              o[d] = od;
            }
            if (hit) {
              const int slot = atomicAdd(ncomp, 1);
              off[3 * slot] = o[0];
              off[3 * slot + 1] = o[1];
              off[3 * slot + 2] = o[2];
              const Quad<T> f = sfq[i];
              window_weights<T, P>(g, coef, nullptr, f.fx, wx + slot * P, nullptr);
              window_weights<T, P>(g, coef, nullptr, f.fy, wy + slot * P, nullptr);
              window_weights<T, P>(g, coef, nullptr, f.fz, wz + slot * P, nullptr);
#pragma unroll
              for (int k = 0; k < P; ++k) wz[slot * P + k] *= f.q;
            }
          }
          __syncthreads();
          // 2. accumulate: one wavefront per particle, lanes over (ix, iy)
          const int nc = *ncomp;
          for (int s = wave; s < nc; s += nwaves) {
            const int ox = off[3 * s], oy = off[3 * s + 1], oz = off[3 * s + 2];
            for (int l = lane; l < P * P; l += 64) {
              const int ix = l % P, iy = l / P;
              int px = ox + ix, py = oy + iy;
              if (g.per[0] && px >= g.G[0]) px -= g.G[0];
              if (g.per[1] && py >= g.G[1]) py -= g.G[1];
              if (px < 0 || px >= ex || py < 0 || py >= ey) continue;
              const T wxy = wx[s * P + ix] * wy[s * P + iy];
#pragma unroll
              for (int iz = 0; iz < P; ++iz) {
                int pz = oz + iz;
                if (g.per[2] && pz >= g.G[2]) pz -= g.G[2];
                if (pz < 0 || pz >= ez) continue;
                atomicAdd(&acc[(pz * TT + py) * TT + px], wxy * wz[s * P + iz]);
              }
            }
          }
          __syncthreads();
          if (threadIdx.x == 0) *ncomp = 0;
          __syncthreads();
        }
      }

  // write the tile once
  T* grid = reinterpret_cast<T*>(b.grid);
  const int n = ex * ey * ez;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int px = e % ex, py = (e / ex) % ey, pz = e / (ex * ey);
    grid[((long long)(z0 + pz) * g.G[1] + (y0 + py)) * g.G[0] + (x0 + px)] = acc[(pz * TT + py) * TT + px];
  }
}

template <typename T>
size_t spread_lds(const GridGeom& g) {
  const int TT = g.tile, P = g.P, m = g.nu + 1, C = g.chunk;
  return sizeof(T) * ((size_t)TT * TT * TT + 3 * C * P + P * m) + sizeof(int) * (3 * C + 4);
}

template <typename T, int P>
static void spread_launch(const GridGeom& g, const EvalBuffers& b, hipStream_t st) {
  const int ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  spread_kernel<T, P><<<dim3(ntiles), dim3(kBlock), spread_lds<T>(g), st>>>(g, b);
}

template <typename T>
static hipError_t spread_dispatch(const GridGeom& g, const EvalBuffers& b, hipStream_t st) {
  switch (g.P) {
    case 2: spread_launch<T, 2>(g, b, st); break;
    case 4: spread_launch<T, 4>(g, b, st); break;
    case 6: spread_launch<T, 6>(g, b, st); break;
    case 8: spread_launch<T, 8>(g, b, st); break;
    case 10: spread_launch<T, 10>(g, b, st); break;
    case 12: spread_launch<T, 12>(g, b, st); break;
    case 14: spread_launch<T, 14>(g, b, st); break;
    case 16: spread_launch<T, 16>(g, b, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t spread_lds_bytes(const GridGeom& g, bool f64) {
  return f64 ? spread_lds<double>(g) : spread_lds<float>(g);
}

hipError_t launch_spread(const GridGeom& g, const EvalBuffers& b, bool f64, hipStream_t st) {
  return f64 ? spread_dispatch<double>(g, b, st) : spread_dispatch<float>(g, b, st);
}

// ---------------------------------------------------------------------------
// Gathering
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void gather_kernel(GridGeom g, EvalBuffers b, T* __restrict__ phi,
                                                        T* __restrict__ force, int out_grad,
                                                        double self_coef) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int t_id = blockIdx.x;
  const int start = b.tile_start[t_id], end = b.tile_start[t_id + 1];
  __shared__ double ewave[kBlock / 64];
  if (start == end) {
    if (threadIdx.x == 0) b.epart[t_id] = 0.0;
    return;
  }
  const int TT = g.tile;
  const int R = TT + P - 1;
  const int tz = t_id / (g.nt[0] * g.nt[1]);
  const int ty = (t_id / g.nt[0]) % g.nt[1];
  const int tx = t_id % g.nt[0];
  const int x0 = tx * TT, y0 = ty * TT, z0 = tz * TT;
  const int m = g.nu + 1;

  const int kChunk = g.chunk;
  T* reg = reinterpret_cast<T*>(smem);                   // R^3
  T* wx = reg + R * R * R;                                // kChunk * P each
  T* wy = wx + kChunk * P;
  T* wz = wy + kChunk * P;
  T* dx = wz + kChunk * P;
  T* dy = dx + kChunk * P;
  T* dz = dy + kChunk * P;
  T* coef = dz + kChunk * P;                              // P*m
  T* dcoef = coef + P * m;                                // P*m
  int* loc = reinterpret_cast<int*>(dcoef + P * m);       // kChunk * 3
  int* pidx = loc + 3 * kChunk;                           // kChunk
  T* pq = reinterpret_cast<T*>(pidx + kChunk);            // kChunk

  const T* wt = reinterpret_cast<const T*>(b.wtab);
  for (int i = threadIdx.x; i < 2 * P * m; i += blockDim.x) coef[i] = wt[i];

  // stage the stencil region [x0 - P/2 + 1, x0 + TT + P/2 - 1] of the grid
  const T* grid = reinterpret_cast<const T*>(b.grid);
  const int rx = x0 - P / 2 + 1, ry = y0 - P / 2 + 1, rz = z0 - P / 2 + 1;
  for (int e = threadIdx.x; e < R * R * R; e += blockDim.x) {
    const int px = e % R, py = (e / R) % R, pz = e / (R * R);
    int gx = rx + px, gy = ry + py, gz = rz + pz;
    bool ok = true;
    if (g.per[0]) { gx %= g.G[0]; if (gx < 0) gx += g.G[0]; } else ok = ok && gx >= 0 && gx < g.G[0];
    if (g.per[1]) { gy %= g.G[1]; if (gy < 0) gy += g.G[1]; } else ok = ok && gy >= 0 && gy < g.G[1];
    if (g.per[2]) { gz %= g.G[2]; if (gz < 0) gz += g.G[2]; } else ok = ok && gz >= 0 && gz < g.G[2];
    reg[e] = ok ? grid[((long long)gz * g.G[1] + gy) * g.G[0] + gx] : (T)0;
  }

  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwaves = blockDim.x / 64;
  const Quad<T>* sfq = reinterpret_cast<const Quad<T>*>(b.s_fq);
  const T sc = (T)g.scale;
  double eacc = 0.0;
  __syncthreads();

  for (int base = start; base < end; base += kChunk) {
    const int cnt = min(kChunk, end - base);
    if (threadIdx.x < cnt) {
      const int i = base + threadIdx.x;
      const int pc = b.s_cell[i];
      loc[3 * threadIdx.x] = (pc & 1023) - x0;
      loc[3 * threadIdx.x + 1] = ((pc >> 10) & 1023) - y0;
      loc[3 * threadIdx.x + 2] = ((pc >> 20) & 1023) - z0;
      pidx[threadIdx.x] = b.s_idx[i];
      const Quad<T> f = sfq[i];
      pq[threadIdx.x] = f.q;
      const int s = threadIdx.x;
      window_weights<T, P>(g, coef, dcoef, f.fx, wx + s * P, dx + s * P);
      window_weights<T, P>(g, coef, dcoef, f.fy, wy + s * P, dy + s * P);
      window_weights<T, P>(g, coef, dcoef, f.fz, wz + s * P, dz + s * P);
    }
    __syncthreads();
    for (int s = wave; s < cnt; s += nwaves) {
      const int cx_ = loc[3 * s], cy = loc[3 * s + 1], cz = loc[3 * s + 2];
      T ph = 0, gx = 0, gy = 0, gz = 0;
      for (int l = lane; l < P * P; l += 64) {
        const int ix = l % P, iy = l / P;
        const T* col = reg + ((long long)cz * R + (cy + iy)) * R + (cx_ + ix);
        T a0 = 0, a1 = 0;
#pragma unroll
        for (int iz = 0; iz < P; ++iz) {
          const T v = col[iz * R * R];
          a0 += v * wz[s * P + iz];
          a1 += v * dz[s * P + iz];
        }
        const T wxy = wx[s * P + ix] * wy[s * P + iy];
        ph += wxy * a0;
        gx += dx[s * P + ix] * wy[s * P + iy] * a0;
        gy += wx[s * P + ix] * dy[s * P + iy] * a0;
        gz += wxy * a1;
      }
      ph = warp_sum(ph);
      gx = warp_sum(gx);
      gy = warp_sum(gy);
      gz = warp_sum(gz);
      if (lane == 0) {
        const int idx = pidx[s];
        const T qv = pq[s];
        const T pv = sc * ph + (T)(self_coef * (double)qv);
        if (phi) phi[idx] = pv;
        if (force) {
          const T f0 = out_grad ? (T)1 : -qv;
          force[3 * idx] = f0 * sc * gx;
          force[3 * idx + 1] = f0 * sc * gy;
          force[3 * idx + 2] = f0 * sc * gz;
        }
        eacc += (double)qv * (double)pv;
      }
    }
    __syncthreads();
  }
  if (lane == 0) ewave[wave] = eacc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += ewave[w];
    b.epart[t_id] = s;
  }
}

template <typename T>
size_t gather_lds(const GridGeom& g) {
  const int R = g.tile + g.P - 1, P = g.P, m = g.nu + 1, C = g.chunk;
  return sizeof(T) * ((size_t)R * R * R + 6 * C * P + 2 * P * m + C) + sizeof(int) * (4 * C);
}

template <typename T, int P>
static void gather_launch(const GridGeom& g, const EvalBuffers& b, T* phi, T* force, int out_grad,
                          double self_coef, hipStream_t st) {
  const int ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  gather_kernel<T, P><<<dim3(ntiles), dim3(kBlock), gather_lds<T>(g), st>>>(g, b, phi, force, out_grad,
                                                                            self_coef);
}

template <typename T>
static hipError_t gather_dispatch(const GridGeom& g, const EvalBuffers& b, void* phi, void* force,
                                  int out_grad, double self_coef, hipStream_t st) {
  T* p = reinterpret_cast<T*>(phi);
  T* f = reinterpret_cast<T*>(force);
  switch (g.P) {
    case 2: gather_launch<T, 2>(g, b, p, f, out_grad, self_coef, st); break;
    case 4: gather_launch<T, 4>(g, b, p, f, out_grad, self_coef, st); break;
    case 6: gather_launch<T, 6>(g, b, p, f, out_grad, self_coef, st); break;
    case 8: gather_launch<T, 8>(g, b, p, f, out_grad, self_coef, st); break;
    case 10: gather_launch<T, 10>(g, b, p, f, out_grad, self_coef, st); break;
    case 12: gather_launch<T, 12>(g, b, p, f, out_grad, self_coef, st); break;
    case 14: gather_launch<T, 14>(g, b, p, f, out_grad, self_coef, st); break;
    case 16: gather_launch<T, 16>(g, b, p, f, out_grad, self_coef, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t gather_lds_bytes(const GridGeom& g, bool f64) {
  return f64 ? gather_lds<double>(g) : gather_lds<float>(g);
}

hipError_t launch_gather(const GridGeom& g, const EvalBuffers& b, bool f64, void* phi, void* force,
                         int out_grad, double self_coef, hipStream_t st) {
  return f64 ? gather_dispatch<double>(g, b, phi, force, out_grad, self_coef, st)
             : gather_dispatch<float>(g, b, phi, force, out_grad, self_coef, st);
}

// E = 1/2 sum of the per-tile partials of q phi, in a fixed order (FP64).
__global__ __launch_bounds__(1024) void energy_kernel(const double* __restrict__ epart, int n,
                                                      double* __restrict__ energy) {
  __shared__ double s[1024];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a += epart[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *energy = 0.5 * s[0];
}

hipError_t launch_energy(const GridGeom& g, const EvalBuffers& b, double* energy, double self_e,
                         hipStream_t st) {
  (void)self_e;
  const int ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  energy_kernel<<<dim3(1), dim3(1024), 0, st>>>(b.epart, ntiles, energy);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Algorithm 3 (free space), FP64
// ---------------------------------------------------------------------------
__global__ void g0p_fill_kernel(cx<double>* buf, int n0, double h, double R) {
  const long long N = (long long)n0 * n0 * n0;
  const double norm = 1.0 / (double)N;  // the inverse transform's 1/n0^3
  const double dk = 2.0 * 3.14159265358979323846 / (n0 * h);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n0), j = (int)((e / n0) % n0), k = (int)(e / ((long long)n0 * n0));
    const int si = i < n0 / 2 ? i : i - n0, sj = j < n0 / 2 ? j : j - n0, sk = k < n0 / 2 ? k : k - n0;
    const double kk = dk * sqrt((double)si * si + (double)sj * sj + (double)sk * sk);
    double v;
    if (kk == 0.0) {
      v = R * R / 2.0;
    } else {
      const double s = sin(R * kk / 2.0) / kk;
      v = 2.0 * s * s;
    }
    buf[e] = cx<double>{v * norm, 0.0};
  }
}

hipError_t launch_g0p_fill(double* buf, int n0, double h, double R, hipStream_t st) {
  g0p_fill_kernel<<<dim3(4096), dim3(kBlock), 0, st>>>(reinterpret_cast<cx<double>*>(buf), n0, h, R);
  return hipGetLastError();
}

// Keep the signed offsets -Mt..Mt-1 of the n0^3 real-space kernel on a (2Mt)^3 grid.
__global__ void g0p_truncate_kernel(const cx<double>* big, int n0, cx<double>* small, int Mt) {
  const int n = 2 * Mt;
  const long long N = (long long)n * n * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)((e / n) % n), k = (int)(e / ((long long)n * n));
    int oi = i < Mt ? i : i - n, oj = j < Mt ? j : j - n, ok = k < Mt ? k : k - n;
    oi = (oi + n0) % n0;
    oj = (oj + n0) % n0;
    ok = (ok + n0) % n0;
    small[e] = big[((long long)ok * n0 + oj) * n0 + oi];
  }
}

hipError_t launch_g0p_truncate(const double* big, int n0, double* small, int Mt, hipStream_t st) {
  g0p_truncate_kernel<<<dim3(4096), dim3(kBlock), 0, st>>>(reinterpret_cast<const cx<double>*>(big), n0,
                                                          reinterpret_cast<cx<double>*>(small), Mt);
  return hipGetLastError();
}

// Octant (Mt+1)^3 of the real, even effective Green's function, index [kx][ky][kz].
template <typename T>
__global__ void g0p_fold_kernel(const cx<double>* full, int Mt, T* table) {
  const int n = 2 * Mt, m = Mt + 1;
  const long long N = (long long)m * m * m;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e % m), j = (int)((e / m) % m), i = (int)(e / ((long long)m * m));
    table[e] = (T)full[((long long)k * n + j) * n + i].re;
  }
}

hipError_t launch_g0p_fold(const double* full, int Mt, void* table, bool f64, hipStream_t st) {
  if (f64)
    g0p_fold_kernel<double><<<dim3(1024), dim3(kBlock), 0, st>>>(reinterpret_cast<const cx<double>*>(full), Mt,
                                                                 reinterpret_cast<double*>(table));
  else
    g0p_fold_kernel<float><<<dim3(1024), dim3(kBlock), 0, st>>>(reinterpret_cast<const cx<double>*>(full), Mt,
                                                                reinterpret_cast<float*>(table));
  return hipGetLastError();
}

}  // namespace se
