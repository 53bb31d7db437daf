// gfx950 pencil transforms of the Spectral Ewald k-space path (Algorithms 1-3
// of Shamshirgar, Bagge, Tornberg, arXiv:1712.04732).
//
// One workgroup transforms B pencils of one length-n class at once: it loads
// them into LDS (zero padding up to n), runs mixed-radix (2,3,4,5,6,7,8,9)
// Stockham stages in place in one LDS buffer (each thread holds its
// butterflies of a stage in registers across a barrier; blocks above 2048
// samples alternate between two buffers instead), and stores the first n_out
// samples (truncation).  Real-to-complex and complex-to-real passes transform two real
// pencils as the real and imaginary parts of one complex pencil.  The fused
// pass runs the forward transform, the scaling of Eq. (scale) and the inverse
// transform of a pencil without leaving LDS.
//
// Addressing: every per-lane offset is kept relative to a per-workgroup base
// held in scalar registers and advanced by additions; offsets are 32-bit
// unless a workgroup's pencils span 4 GiB (then 64-bit).  LDS addresses are
// 32-bit and butterfly strides are uniform, so a butterfly input or output
// costs one vector add.
#include "se_device.h"

namespace se {

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
  // a_r = v_r + v_{R-r}, b_r = v_r - v_{R-r}, kept in v_r and v_{R-r}
  cx<T> x0 = v[0];
#pragma unroll
  for (int r = 1; r <= H; ++r) {
    const cx<T> a = v[r] + v[R - r], b = v[r] - v[R - r];
    v[r] = a;
    v[R - r] = b;
    x0 = x0 + a;
  }
  // outputs m and R - m share the cosine sum A_m and the sine sum B_m:
  // X_m = A_m + sign i B_m, X_{R-m} = A_m - sign i B_m
  cx<T> out[R];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    cx<T> A = v[0], Bs = {0, 0};
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      const int j = (r * m) % R;
      A = A + cscale(v[r], (T)OddRoots<R>::c[j]);
      Bs = Bs + cscale(v[R - r], (T)OddRoots<R>::s[j]);
    }
    const cx<T> iB = mul_si(Bs, sign);
    out[m] = A + iB;
    out[R - m] = A - iB;
  }
  v[0] = x0;
#pragma unroll
  for (int m = 1; m < R; ++m) v[m] = out[m];
}

// Composite radix R = R1 R2 (6 = 2 x 3, 9 = 3 x 3) in registers: with
// k = m + R2 q, X_k = sum_j exp(sign 2 pi i j q / R1) [exp(sign 2 pi i j m / R)
// A_j(m)], where A_j is the length-R2 DFT of v_j, v_{j+R1}, ...  One stage of
// radix R replaces two stages of radices R1 and R2 (one LDS round trip and
// one barrier fewer).
template <int R>
struct MixedRoots;
template <>
struct MixedRoots<6> {   // exp(2 pi i t / 6), t = j m for j < 2, m < 3
  static constexpr int R1 = 2, R2 = 3;
  static constexpr double c[3] = {1.0, 0.5, -0.5};
  static constexpr double s[3] = {0.0, 0.86602540378443864676, 0.86602540378443864676};
};
template <>
struct MixedRoots<9> {   // exp(2 pi i t / 9), t = j m for j, m < 3
  static constexpr int R1 = 3, R2 = 3;
  static constexpr double c[5] = {1.0, 0.76604444311897803520, 0.17364817766693034885, 0.0,
                                  -0.93969262078590838405};
  static constexpr double s[5] = {0.0, 0.64278760968653932632, 0.98480775301220805936, 0.0,
                                  0.34202014332566873304};
};

template <typename T, int R>
__device__ __forceinline__ void dft(cx<T>* v, int sign);

template <typename T, int R>
__device__ __forceinline__ void dft_mixed(cx<T>* v, int sign) {
  constexpr int R1 = MixedRoots<R>::R1, R2 = MixedRoots<R>::R2;
  cx<T> a[R1][R2];
#pragma unroll
  for (int j = 0; j < R1; ++j) {
#pragma unroll
    for (int r = 0; r < R2; ++r) a[j][r] = v[j + R1 * r];
    dft<T, R2>(a[j], sign);
#pragma unroll
    for (int m = 1; m < R2; ++m)
      if (j > 0) {
        const int t = j * m;
        a[j][m] = cmul(a[j][m], cx<T>{(T)MixedRoots<R>::c[t], (T)(sign * MixedRoots<R>::s[t])});
      }
  }
#pragma unroll
  for (int m = 0; m < R2; ++m) {
    cx<T> b[R1];
#pragma unroll
    for (int j = 0; j < R1; ++j) b[j] = a[j][m];
    dft<T, R1>(b, sign);
#pragma unroll
    for (int q = 0; q < R1; ++q) v[m + R2 * q] = b[q];
  }
}

template <typename T, int R>
__device__ __forceinline__ void dft(cx<T>* v, int sign) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 4) dft4(v, sign);
  else if constexpr (R == 8) dft8(v, sign);
  else if constexpr (R == 6 || R == 9) dft_mixed<T, R>(v, sign);
  else dft_odd<T, R>(v, sign);
}


// LDS views.  Arithmetic on these pointers is 32-bit.
template <typename T>
using lds = __attribute__((address_space(3))) T;

template <typename T>
__device__ __forceinline__ cx<T> lget(const lds<vec2<T>>* p, int i) {
  const vec2<T> v = p[i];
  return cx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void lput(lds<vec2<T>>* p, int i, cx<T> v) {
  p[i] = vec2<T>{v.re, v.im};
}

// Global loads and stores at a byte offset from a base pointer.  With a
// uniform base and a 32-bit offset the compiler addresses them as scalar base
// plus vector offset.
template <typename V, typename OFF>
__device__ __forceinline__ V gload(const void* base, OFF off) {
  return *(const __attribute__((address_space(1))) V*)((const __attribute__((address_space(1))) char*)base + off);
}
template <typename V, typename OFF>
__device__ __forceinline__ void gstore(void* base, OFF off, V v) {
  *(__attribute__((address_space(1))) V*)((__attribute__((address_space(1))) char*)base + off) = v;
}

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Reciprocal for the quotients fdiv(a, .) of the transforms, whose
// dividends stay below kFftCap = 2^13: the hardware reciprocal (relative
// error below 2^-22) and the product's rounding move (a + 1/2)/d by less than
// 2^13 2^-21 / d = 2^-8 / d, far inside the 1/(2d) that separates it from an
// integer, so truncation is still exact.
__device__ __forceinline__ float quot_recip(int d) { return __builtin_amdgcn_rcpf((float)d); }
// The same for a divisor uniform over the workgroup, kept in a scalar register.
__device__ __forceinline__ float quot_recip_u(int d) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(quot_recip(d))));
}

// One Stockham stage from src to dst over F interleaved pencils stored
// sample-major with pitch Bp (sample t of pencil p at t Bp + p).  Slot e holds
// butterfly j = e div F of pencil p = e mod F; butterfly j reads samples j + r n/R, multiplies input r by the twiddle
// exp(sign 2 pi i r k/(Ns R)) = tw[r k tws] (k = j mod Ns, tws = n/(Ns R)),
// and writes outputs (j div Ns) Ns R + k + r Ns.  The first stage (Ns = 1)
// has no twiddles.
template <typename T, int R, bool FIRST, int SIGN>
__device__ __forceinline__ void fft_stage(const lds<vec2<T>>* __restrict__ src, lds<vec2<T>>* __restrict__ dst,
                                          const lds<vec2<T>>* __restrict__ tw, int n, int Ns, int tws, int F,
                                          int Bp) {
  const int nb = n / R;
  const int total = __mul24(nb, F);
  const float inv_f = quot_recip_u(F);
  const int sstr = nb * Bp;   // between the inputs of a butterfly
  const int dstr = Ns * Bp;   // between its outputs
  const int nsr = Ns * R;
  const float inv_ns = quot_recip(Ns);
  for (int e = threadIdx.x; e < total; e += kFftBlock) {
    const int j = fdiv(e, inv_f), p = e - __mul24(j, F);
    const lds<vec2<T>>* s = src + (__mul24(j, Bp) + p);
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lget<T>(s, r * sstr);
    int base;
    if constexpr (FIRST) {
      base = __mul24(j, R);
    } else {
      const int jq = fdiv(j, inv_ns), k = j - __mul24(jq, Ns);
      const int kt = __mul24(k, tws);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = lget<T>(tw, r * kt);   // r k tws < R Ns tws = n
        if constexpr (SIGN > 0) w.im = -w.im;
        v[r] = cmul(v[r], w);
      }
      base = __mul24(jq, nsr) + k;
    }
    dft<T, R>(v, SIGN);
    lds<vec2<T>>* d = dst + (__mul24(base, Bp) + p);
#pragma unroll
    for (int r = 0; r < R; ++r) lput<T>(d, r * dstr, v[r]);
  }
}

template <typename T, bool FIRST, int SIGN>
__device__ __forceinline__ void fft_stage_r(int R, const lds<vec2<T>>* src, lds<vec2<T>>* dst,
                                            const lds<vec2<T>>* tw, int n, int Ns, int tws, int F, int Bp) {
  switch (R) {
    case 2: fft_stage<T, 2, FIRST, SIGN>(src, dst, tw, n, Ns, tws, F, Bp); break;
    case 3: fft_stage<T, 3, FIRST, SIGN>(src, dst, tw, n, Ns, tws, F, Bp); break;
    case 4: fft_stage<T, 4, FIRST, SIGN>(src, dst, tw, n, Ns, tws, F, Bp); break;
    case 5: fft_stage<T, 5, FIRST, SIGN>(src, dst, tw, n, Ns, tws, F, Bp); break;
    case 6: fft_stage<T, 6, FIRST, SIGN>(src, dst, tw, n, Ns, tws, F, Bp); break;
    case 7: fft_stage<T, 7, FIRST, SIGN>(src, dst, tw, n, Ns, tws, F, Bp); break;
    case 9: fft_stage<T, 9, FIRST, SIGN>(src, dst, tw, n, Ns, tws, F, Bp); break;
    default: fft_stage<T, 8, FIRST, SIGN>(src, dst, tw, n, Ns, tws, F, Bp); break;
  }
}

// All stages of class C (radices packed 4 bits per stage, first stage lowest),
// alternating between the two buffers; returns the buffer holding the result.
template <typename T, int SIGN>
__device__ __forceinline__ lds<vec2<T>>* fft_run(lds<vec2<T>>* b0, lds<vec2<T>>* b1, const lds<vec2<T>>* tw,
                                                 const FftClass& C, int F, int Bp) {
  lds<vec2<T>>* src = b0;
  lds<vec2<T>>* dst = b1;
  const int n = C.n, nst = C.nst;
  unsigned long long radices = C.radpack;
  int Ns = 1, rem = n;   // rem = n / Ns
  for (int s = 0; s < nst; ++s) {
    const int R = (int)(radices & 15u);
    radices >>= 4;
    const int tws = rem / R;
    if (s == 0) fft_stage_r<T, true, SIGN>(R, src, dst, tw, n, Ns, tws, F, Bp);
    else fft_stage_r<T, false, SIGN>(R, src, dst, tw, n, Ns, tws, F, Bp);
    __syncthreads();
    lds<vec2<T>>* tmp = src;
    src = dst;
    dst = tmp;
    Ns *= R;
    rem = tws;
  }
  return src;
}

// The same stage in place: every thread first reads and transforms all its
// butterflies (at most kFftIpIters(R) of them, held in registers; the
// planner keeps (n / R) B within kFftIpIters(R) kFftBlock), then, after a
// barrier, writes them back over the inputs.
template <typename T, int R, bool FIRST, int SIGN>
__device__ __forceinline__ void fft_stage_ip(lds<vec2<T>>* buf, const lds<vec2<T>>* __restrict__ tw, int n, int Ns,
                                             int tws, int F, int Bp) {
  constexpr int IT = kFftIpIters(R);
  const int nb = n / R;
  const int total = __mul24(nb, F);
  const float inv_f = quot_recip_u(F);
  const int sstr = nb * Bp;
  const int dstr = Ns * Bp;
  const int nsr = Ns * R;
  const float inv_ns = quot_recip(Ns);
  cx<T> v[IT][R];
  int dofs[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * kFftBlock;
    dofs[it] = -1;
    if (e < total) {
      const int j = fdiv(e, inv_f), p = e - __mul24(j, F);
      const lds<vec2<T>>* s = buf + (__mul24(j, Bp) + p);
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = lget<T>(s, r * sstr);
      int base;
      if constexpr (FIRST) {
        base = __mul24(j, R);
      } else {
        const int jq = fdiv(j, inv_ns), k = j - __mul24(jq, Ns);
        const int kt = __mul24(k, tws);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = lget<T>(tw, r * kt);
          if constexpr (SIGN > 0) w.im = -w.im;
          v[it][r] = cmul(v[it][r], w);
        }
        base = __mul24(jq, nsr) + k;
      }
      dft<T, R>(v[it], SIGN);
      dofs[it] = __mul24(base, Bp) + p;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it)
    if (dofs[it] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) lput<T>(buf, dofs[it] + r * dstr, v[it][r]);
    }
  __syncthreads();
}

template <typename T, bool FIRST, int SIGN>
__device__ __forceinline__ void fft_stage_ip_r(int R, lds<vec2<T>>* buf, const lds<vec2<T>>* tw, int n, int Ns,
                                               int tws, int F, int Bp) {
  switch (R) {
    case 2: fft_stage_ip<T, 2, FIRST, SIGN>(buf, tw, n, Ns, tws, F, Bp); break;
    case 3: fft_stage_ip<T, 3, FIRST, SIGN>(buf, tw, n, Ns, tws, F, Bp); break;
    case 4: fft_stage_ip<T, 4, FIRST, SIGN>(buf, tw, n, Ns, tws, F, Bp); break;
    case 5: fft_stage_ip<T, 5, FIRST, SIGN>(buf, tw, n, Ns, tws, F, Bp); break;
    case 6: fft_stage_ip<T, 6, FIRST, SIGN>(buf, tw, n, Ns, tws, F, Bp); break;
    case 7: fft_stage_ip<T, 7, FIRST, SIGN>(buf, tw, n, Ns, tws, F, Bp); break;
    case 9: fft_stage_ip<T, 9, FIRST, SIGN>(buf, tw, n, Ns, tws, F, Bp); break;
    default: fft_stage_ip<T, 8, FIRST, SIGN>(buf, tw, n, Ns, tws, F, Bp); break;
  }
}

// All stages of class C in place in buf.
template <typename T, int SIGN>
__device__ __forceinline__ void fft_run_ip(lds<vec2<T>>* buf, const lds<vec2<T>>* tw, const FftClass& C, int F,
                                           int Bp) {
  const int n = C.n, nst = C.nst;
  unsigned long long radices = C.radpack;
  int Ns = 1, rem = n;
  for (int s = 0; s < nst; ++s) {
    const int R = (int)(radices & 15u);
    radices >>= 4;
    const int tws = rem / R;
    if (s == 0) fft_stage_ip_r<T, true, SIGN>(R, buf, tw, n, Ns, tws, F, Bp);
    else fft_stage_ip_r<T, false, SIGN>(R, buf, tw, n, Ns, tws, F, Bp);
    Ns *= R;
    rem = tws;
  }
}

__device__ __forceinline__ int fold_index(int i, int n) { return i <= n - i ? i : n - i; }

// The factors of Eq. (scale) that depend only on the pencil (b0, b1): the
// separable vectors of the two pencil directions and the pencil's part of the
// table or |k|^2 index.
template <typename T>
struct ScaleRow {
  T s;     // sA[b0] sB[b1]
  T k2;    // kA[b0] + kB[b1]            (G_INVSQ)
  int g;   // table offset of the pencil (G_TAB2, G_TAB3)
};

template <typename T>
__device__ __forceinline__ ScaleRow<T> scale_row(const FftClass& C, int b0, int b1) {
  ScaleRow<T> r;
  r.s = gld((const T*)C.sA)[b0 + C.offA] * gld((const T*)C.sB)[b1 + C.offB];
  r.k2 = 0;
  r.g = 0;
  const int i0 = C.fold0 ? fold_index(b0, C.fold0) : b0;
  if (C.gmode == G_INVSQ) r.k2 = gld((const T*)C.kA)[b0 + C.offA] + gld((const T*)C.kB)[b1 + C.offB];
  else if (C.gmode == G_TAB2) r.g = i0;
  else if (C.gmode == G_TAB3) r.g = fold_index(b1, C.fold1) * C.gd0 + i0;
  return r;
}

// Tables store the pencil index b0 fastest, so neighbouring lanes (neighbouring
// pencils) read neighbouring entries: G_TAB2 [t][b0], G_TAB3 [t][b1][b0].
template <typename T>
__device__ __forceinline__ T scale_at(const FftClass& C, const ScaleRow<T>& r, int t) {
  const T s = r.s * gld((const T*)C.sC)[t];
  const auto gt = gld((const T*)C.gtab);
  switch (C.gmode) {
    case G_INVSQ: {
      const T k2 = r.k2 + gld((const T*)C.kC)[t];
      return k2 > (T)0 ? s / k2 : (T)0;
    }
    case G_TAB1:
      return s * gt[t];
    case G_TAB2:
      return s * gt[fold_index(t, C.fold2) * C.gd0 + r.g];
    case G_TAB3:
      return s * gt[fold_index(t, C.fold2) * (C.gd1 * C.gd0) + r.g];
    default:
      return s;
  }
}

// The scaling of Eq. (scale) over the samples t = t0, t0 + dt, ... of pencil
// p in res (sample-major, pitch Bp), the same arithmetic as scale_at.  The
// table entries of up to kScaleRound samples are loaded before any is used,
// so a thread waits for one round of loads rather than one per sample.
constexpr int kScaleRound = kFftInplaceCap / kFftBlock;

template <typename T, int GM>
__device__ __forceinline__ void scale_pencil(const FftClass& C, const ScaleRow<T>& row, lds<vec2<T>>* res, int p,
                                             int t0, int dt, int n, int Bp) {
  const T* sC = (const T*)C.sC;
  const T* aux = GM == G_INVSQ ? (const T*)C.kC : (const T*)C.gtab;
  for (int tb = t0; tb < n; tb += kScaleRound * dt) {
    T a[kScaleRound], b[kScaleRound];
#pragma unroll
    for (int i = 0; i < kScaleRound; ++i) {
      const int t = tb + i * dt;
      a[i] = (T)0;
      b[i] = (T)0;
      if (t < n) {
        a[i] = gld(sC)[t];
        if constexpr (GM == G_INVSQ || GM == G_TAB1) b[i] = gld(aux)[t];
        else if constexpr (GM == G_TAB2) b[i] = gld(aux)[fold_index(t, C.fold2) * C.gd0 + row.g];
        else if constexpr (GM == G_TAB3) b[i] = gld(aux)[fold_index(t, C.fold2) * (C.gd1 * C.gd0) + row.g];
      }
    }
#pragma unroll
    for (int i = 0; i < kScaleRound; ++i) {
      const int t = tb + i * dt;
      if (t < n) {
        const T s = row.s * a[i];
        T f;
        if constexpr (GM == G_INVSQ) {
          const T k2 = row.k2 + b[i];
          f = k2 > (T)0 ? s / k2 : (T)0;
        } else if constexpr (GM == G_NONE) {
          f = s;
        } else {
          f = s * b[i];
        }
        const int l = __mul24(t, Bp) + p;
        lput<T>(res, l, cscale(lget<T>(res, l), f));
      }
    }
  }
}

// The slots one thread visits when a workgroup streams an n x B block of
// pencil samples: slots tid, tid + kFftBlock, ...  Slot order is pencil-major
// (p = e div n, t = e mod n) when the transform direction is contiguous in
// memory (TF) and sample-major (t = e div B, p = e mod B) otherwise, so that
// neighbouring lanes touch neighbouring addresses.  The thread tracks the
// sample t, the pencil p, a global byte offset g = p gs0 + t gst and an LDS
// index l = t lt + p lp, all advanced by additions: a step of kFftBlock slots
// moves the slow index (p if TF, else t) by q and the fast one by r, and a
// fast index that passes its limit (n if TF, else B) wraps into the slow one.
template <bool TF, typename OFF>
struct SlotWalk {
  int lim, q, r;
  OFF dg, dgw;
  int dl, dlw;
  int t, p;
  OFF g;
  int l;

  __device__ __forceinline__ SlotWalk(int n, int B, OFF gs0, OFF gst, int lt, int lp) {
    const int tid = threadIdx.x;
    lim = TF ? n : B;
    const float inv = quot_recip(lim);
    // uniform: kept in scalar registers
    q = rfl(fdiv(kFftBlock, inv));
    r = kFftBlock - q * lim;
    const int slow = fdiv(tid, inv), fast = tid - slow * lim;
    if constexpr (TF) {
      p = slow;
      t = fast;
      dg = (OFF)r * gst + (OFF)q * gs0;
      dgw = gs0 - (OFF)n * gst;
      dl = r * lt + q * lp;
      dlw = lp - n * lt;
    } else {
      t = slow;
      p = fast;
      dg = (OFF)r * gs0 + (OFF)q * gst;
      dgw = gst - (OFF)B * gs0;
      dl = r * lp + q * lt;
      dlw = lt - B * lp;
    }
    g = (OFF)p * gs0 + (OFF)t * gst;
    l = t * lt + p * lp;
  }
  __device__ __forceinline__ void step() {
    int& fast = TF ? t : p;
    int& slow = TF ? p : t;
    fast += r;
    slow += q;
    g += dg;
    l += dl;
    const bool w = fast >= lim;
    fast = w ? fast - lim : fast;
    slow = w ? slow + 1 : slow;
    g = w ? g + dgw : g;
    l = w ? l + dlw : l;
  }
};

// A real pencil pair (a, b) shares one complex transform z = a + i b.  Forward:
// A_k = (Z_k + conj Z_{n-k})/2 and B_k = (Z_k - conj Z_{n-k})/(2i).  Inverse:
// the half spectra of a and b, Hermitian-extended, combine to Z = A + i B, whose
// transform holds a in the real and b in the imaginary part.
template <typename T>
__device__ __forceinline__ cx<T> split_pair(cx<T> z, cx<T> zn, int odd) {
  return odd ? cx<T>{(T)0.5 * (z.im + zn.im), (T)0.5 * (zn.re - z.re)}
             : cx<T>{(T)0.5 * (z.re + zn.re), (T)0.5 * (z.im - zn.im)};
}

constexpr int kSlotsInFlight = 8;   // global loads in flight per thread

// Load phase: pencils p < cnt of the work item into buf (sample-major, pitch
// Bp), zero padded from n_in to n; twiddles into tw.  C2R reads the stored
// half spectrum (t <= n/2) and extends it by Hermitian symmetry.
template <typename T, int KIND, bool TF, typename OFF>
__device__ __forceinline__ void fft_load(const FftClass& C, int b0s, int b1, int cnt, int B, int pair, int Bp,
                                         lds<vec2<T>>* buf, lds<vec2<T>>* tw) {
  constexpr int U = kSlotsInFlight;
  using V2 = vec2<T>;
  const int n = C.n;
  // twiddle table: the first kFftBlock entries travel with the first round
  const bool has_tw = (int)threadIdx.x < n;
  V2 tw0 = V2{0, 0};
  if (has_tw) tw0 = gld(reinterpret_cast<const V2*>(C.tw))[threadIdx.x];
  auto put_twiddles = [&]() {
    if (has_tw) tw[threadIdx.x] = tw0;
    for (int i = threadIdx.x + kFftBlock; i < n; i += kFftBlock) tw[i] = gld(reinterpret_cast<const V2*>(C.tw))[i];
  };
  if constexpr (KIND == K_C2R) {
    // slots (t, complex pencil c) over the stored half t <= n/2, c < B / 2^pair:
    // pencils a = 2c, b = 2c + 1 (paired) or a = c.  Each stored bin is read
    // once and gives, by Hermitian symmetry, Z_t = A_t + i B_t and, for
    // 0 < t < n - t, Z_{n-t} = conj(A_t) + i conj(B_t).
    constexpr OFF esz = 2 * sizeof(T);
    const int F = pair ? B >> 1 : B;
    const char* base = (const char*)C.in + ((long long)b0s * C.in_s0 + (long long)b1 * C.in_s1) * (long long)esz;
    const OFF gs0 = (OFF)C.in_s0 * esz, gst = (OFF)C.in_st * esz;
    const OFF gsp = gs0 << pair;
    const int nh = (n >> 1) + 1, total = nh * F;
    SlotWalk<TF, OFF> w(nh, F, gsp, (OFF)0, Bp, 1);   // g tracks the pencil part only
    for (int e0 = 0; e0 < total; e0 += U * kFftBlock) {
      V2 va[U], vb[U];
      int lw[U], tt[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        va[u] = V2{0, 0};
        vb[u] = V2{0, 0};
        const int pa = w.p << pair;
        const OFF go = w.g + (TF ? (OFF)w.t * esz : (OFF)w.t * gst);
        if (w.t < nh && pa < cnt) {
          va[u] = gload<V2>(base, go);
          if (pair && pa + 1 < cnt) vb[u] = gload<V2>(base, go + gs0);
        }
        lw[u] = (w.t < nh && w.p < F) ? w.l : -1;
        tt[u] = w.t;
        w.step();
      }
      if (e0 == 0) put_twiddles();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (lw[u] < 0) continue;
        const V2 a = va[u], b = vb[u];
        lput<T>(buf, lw[u], cx<T>{a.x - b.y, a.y + b.x});
        const int t = tt[u];
        if (t > 0 && t < n - t) lput<T>(buf, lw[u] + __mul24(n - 2 * t, Bp), cx<T>{a.x + b.y, b.x - a.y});
      }
    }
  } else {
    // slots (t, pencil p), p < B; a paired real pass packs pencil p into
    // component p & 1 of complex pencil p / 2 (LDS float index 2 t Bp + p)
    constexpr bool RIN = (KIND == K_R2C);
    constexpr OFF esz = RIN ? sizeof(T) : 2 * sizeof(T);
    const char* base = (const char*)C.in + ((long long)b0s * C.in_s0 + (long long)b1 * C.in_s1) * (long long)esz;
    const OFF gs0 = (OFF)C.in_s0 * esz, gst = (OFF)C.in_st * esz;
    const int total = n * B, n_in = C.n_in;
    SlotWalk<TF, OFF> w(n, B, gs0, gst, pair ? 2 * Bp : Bp, 1);
    lds<T>* fbuf = reinterpret_cast<lds<T>*>(buf);
    for (int e0 = 0; e0 < total; e0 += U * kFftBlock) {
      cx<T> v[U];
      int lw[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = cx<T>{0, 0};
        if (w.p < cnt && w.t < n_in) {
          if constexpr (RIN) {
            v[u].re = gload<T>(base, w.g);
          } else {
            const V2 a = gload<V2>(base, w.g);
            v[u] = cx<T>{a.x, a.y};
          }
        }
        lw[u] = (w.t < n && w.p < B) ? w.l : -1;
        w.step();
      }
      if (e0 == 0) put_twiddles();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (lw[u] < 0) continue;
        if (RIN && pair) fbuf[lw[u]] = v[u].re;
        else lput<T>(buf, lw[u], v[u]);
      }
    }
  }
}

// Store phase: the first n_out samples of pencils p < cnt from res.
template <typename T, int KIND, bool TF, typename OFF>
__device__ __forceinline__ void fft_store(const FftClass& C, int b0s, int b1, int cnt, int B, int pair, int Bp,
                                          const lds<vec2<T>>* res) {
  constexpr int U = kSlotsInFlight;
  constexpr bool ROUT = (KIND == K_C2R);
  constexpr OFF esz = ROUT ? sizeof(T) : 2 * sizeof(T);
  const int n = C.n, nout = C.n_out;
  char* base = (char*)C.out + ((long long)b0s * C.out_s0 + (long long)b1 * C.out_s1) * (long long)esz;
  const OFF gs0 = (OFF)C.out_s0 * esz, gst = (OFF)C.out_st * esz;
  const int total = nout * B;
  // LDS index of slot (t, p): complex t Bp + p; for the real passes the float
  // index 2 t Bp + p (paired) or 2 (t Bp + p) (single pencil, C2R)
  const int lt = (KIND == K_R2C || KIND == K_C2R) ? 2 * Bp : Bp;
  const int lp = (KIND == K_C2R && !pair) ? 2 : 1;
  SlotWalk<TF, OFF> w(nout, B, gs0, gst, lt, lp);
  const lds<T>* fres = reinterpret_cast<const lds<T>*>(res);
  for (int e0 = 0; e0 < total; e0 += U * kFftBlock) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (w.p < cnt && w.t < nout) {
        if constexpr (KIND == K_C2R) {
          gstore<T>(base, w.g, fres[w.l]);
        } else if constexpr (KIND == K_R2C) {
          cx<T> v;
          if (pair) {
            const int lc = w.l >> 1;                  // t Bp + p / 2
            const int tn = w.t == 0 ? 0 : n - w.t;
            v = split_pair(lget<T>(res, lc), lget<T>(res, lc + __mul24(tn - w.t, Bp)), w.p & 1);
          } else {
            v = lget<T>(res, w.l >> 1);               // float index 2 (t Bp + p) for B = 1
          }
          gstore<vec2<T>>(base, w.g, vec2<T>{v.re, v.im});
        } else {
          const cx<T> v = lget<T>(res, w.l);
          gstore<vec2<T>>(base, w.g, vec2<T>{v.re, v.im});
        }
      }
      w.step();
    }
  }
}

// One work item: pencils b0s .. b0s + cnt - 1 at b1 of class cls of pass P.
template <typename T, int KIND, typename OFF>
__device__ __forceinline__ void stage_fft(const FftPass& P, int cls, int b0s, int b1, int cnt,
                                          lds<unsigned char>* smem) {
  constexpr bool REAL = (KIND == K_R2C || KIND == K_C2R);
  const FftClass& C = P.cls[cls];
  const int n = C.n, B = P.B;
  // real passes with B >= 2 (B even) run B/2 complex transforms of pencil pairs
  const int pair = (REAL && B > 1) ? 1 : 0;
  const int F = pair ? B >> 1 : B, Bp = F + 1;
  const bool ip = P.inplace;
  lds<vec2<T>>* tw = reinterpret_cast<lds<vec2<T>>*>(smem);
  lds<vec2<T>>* buf = tw + P.nmax;
  lds<vec2<T>>* buf2 = buf + P.nmax * Bp;   // only if not in place

  if (C.in_st == 1) fft_load<T, KIND, true, OFF>(C, b0s, b1, cnt, B, pair, Bp, buf, tw);
  else fft_load<T, KIND, false, OFF>(C, b0s, b1, cnt, B, pair, Bp, buf, tw);
  __syncthreads();

  constexpr int SIGN = (KIND == K_C2C_INV || KIND == K_C2R) ? +1 : -1;
  lds<vec2<T>>* res = buf;
  if (ip) fft_run_ip<T, SIGN>(buf, tw, C, F, Bp);
  else res = fft_run<T, SIGN>(buf, buf2, tw, C, F, Bp);

  if constexpr (KIND == K_FUSED || KIND == K_FUSED_D) {
    // scaling step, Eq. (scale), on the spectrum of each pencil: thread
    // (t0, p), tid = t0 B + p, takes samples t0, t0 + dt, ... of pencil p,
    // dt = kFftBlock div B (the last kFftBlock mod B threads idle)
    const float inv_b = quot_recip(B);
    int t = fdiv(threadIdx.x, inv_b);
    const int p = threadIdx.x - t * B;
    const int dt = rfl(fdiv(kFftBlock, inv_b)), dl = dt * Bp;
    if (p < cnt && t < dt) {
      const ScaleRow<T> row = scale_row<T>(C, b0s + p, b1);
      if constexpr (KIND == K_FUSED) {
        switch (C.gmode) {
          case G_INVSQ: scale_pencil<T, G_INVSQ>(C, row, res, p, t, dt, n, Bp); break;
          case G_TAB1: scale_pencil<T, G_TAB1>(C, row, res, p, t, dt, n, Bp); break;
          case G_TAB2: scale_pencil<T, G_TAB2>(C, row, res, p, t, dt, n, Bp); break;
          case G_TAB3: scale_pencil<T, G_TAB3>(C, row, res, p, t, dt, n, Bp); break;
          default: scale_pencil<T, G_NONE>(C, row, res, p, t, dt, n, Bp); break;
        }
      } else {
        // force method 2 (Section 7.2): the scaling times i k_d; k_d is a
        // pencil constant for the A and B directions and varies along the
        // pencil (z) otherwise
        const int d = P.deriv;
        const bool along = d != C.dirA && d != C.dirB;
        const T kp = d == C.dirA ? gld((const T*)C.dA)[b0s + p + C.offA]
                                 : (d == C.dirB ? gld((const T*)C.dB)[b1 + C.offB] : (T)0);
        for (int l = __mul24(t, Bp) + p; t < n; t += dt, l += dl) {
          const T k = along ? gld((const T*)C.dC)[t] : kp;
          const cx<T> v = cscale(lget<T>(res, l), scale_at<T>(C, row, t) * k);
          lput<T>(res, l, cx<T>{-v.im, v.re});
        }
      }
    }
    __syncthreads();
    if (ip) fft_run_ip<T, +1>(buf, tw, C, F, Bp);
    else res = fft_run<T, +1>(res, res == buf ? buf2 : buf, tw, C, F, Bp);
  }

  if (C.out_st == 1) fft_store<T, KIND, true, OFF>(C, b0s, b1, cnt, B, pair, Bp, res);
  else fft_store<T, KIND, false, OFF>(C, b0s, b1, cnt, B, pair, Bp, res);
}

// The work record {class, b0 start, b1, count}, the same for the whole
// workgroup (scalar loads).
__device__ __forceinline__ int4 work_record(const int4* rec, int item) {
  const auto p = gld(reinterpret_cast<const int*>(rec)) + 4 * item;
  return make_int4(rfl(p[0]), rfl(p[1]), rfl(p[2]), rfl(p[3]));
}

// FP32 transforms are bound by the latency of their load and store phases:
// capping their registers at 72 (no spills) lets 7 workgroups share a CU
// instead of 5-6.  FP64 transforms, and the 64-bit-offset variants, would
// spill under the cap and keep the compiler's choice.
template <typename T, typename OFF>
constexpr int kFftMinWaves = sizeof(T) == 4 && sizeof(OFF) == 4 ? 7 : 1;

template <typename T, int KIND, typename OFF>
__global__ __launch_bounds__(kFftBlock, (kFftMinWaves<T, OFF>)) void fft_kernel(const FftPass P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 r = work_record(P.items, work_item(P.xcd));
  stage_fft<T, KIND, OFF>(P, r.x, r.y, r.z, r.w, (lds<unsigned char>*)smem);
}

// One transform kind of one transform stage of a batch: block b takes record
// b of the (stage, kind) list, {system * 4 + class, b0 start, b1, count}, so a
// workgroup finds its system and pencils with one scalar load.
template <typename T, int KIND, typename OFF>
__global__ __launch_bounds__(kFftBlock, (kFftMinWaves<T, OFF>)) void batch_fft_kernel(const SysDesc* __restrict__ sys,
                                                              const int4* __restrict__ rec, int pass, int xcd) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 r = work_record(rec, work_item(xcd));
  stage_fft<T, KIND, OFF>(sys[r.x >> 2].pass[pass], r.x & 3, r.y, r.z, r.w, (lds<unsigned char>*)smem);
}

size_t fft_lds_bytes(const FftPass& p, bool f64) {
  const size_t c = f64 ? 16 : 8;
  const size_t nbuf = p.inplace ? 1 : 2;
  // complex transforms per block: B, or B / 2 pencil pairs for the real passes
  const bool pair = (p.kind == K_R2C || p.kind == K_C2R) && p.B > 1;
  return c * ((size_t)p.nmax + nbuf * ((size_t)(pair ? p.B / 2 : p.B) + 1) * p.nmax);
}

template <typename T, typename OFF>
static void launch_fft_t(const FftPass& p, hipStream_t st) {
  const size_t lds = fft_lds_bytes(p, sizeof(T) == 8);
  const dim3 grid(p.nitems), block(kFftBlock);
  switch (p.kind) {
    case K_C2C_FWD: fft_kernel<T, K_C2C_FWD, OFF><<<grid, block, lds, st>>>(p); break;
    case K_C2C_INV: fft_kernel<T, K_C2C_INV, OFF><<<grid, block, lds, st>>>(p); break;
    case K_R2C: fft_kernel<T, K_R2C, OFF><<<grid, block, lds, st>>>(p); break;
    case K_C2R: fft_kernel<T, K_C2R, OFF><<<grid, block, lds, st>>>(p); break;
    case K_FUSED_D: fft_kernel<T, K_FUSED_D, OFF><<<grid, block, lds, st>>>(p); break;
    default: fft_kernel<T, K_FUSED, OFF><<<grid, block, lds, st>>>(p); break;
  }
}

hipError_t launch_fft(const FftPass& p, bool f64, hipStream_t st) {
  if (p.nitems <= 0) return hipSuccess;
  using W = unsigned long long;
  if (f64) p.wide ? launch_fft_t<double, W>(p, st) : launch_fft_t<double, unsigned>(p, st);
  else p.wide ? launch_fft_t<float, W>(p, st) : launch_fft_t<float, unsigned>(p, st);
  return hipGetLastError();
}

template <typename T, typename OFF>
static void launch_batch_fft_t(int kind, const SysDesc* sys, const int4* rec, int pass, int nitems, size_t lds,
                               int xcd, hipStream_t st) {
  const dim3 grid(nitems), block(kFftBlock);
  switch (kind) {
    case K_C2C_FWD: batch_fft_kernel<T, K_C2C_FWD, OFF><<<grid, block, lds, st>>>(sys, rec, pass, xcd); break;
    case K_C2C_INV: batch_fft_kernel<T, K_C2C_INV, OFF><<<grid, block, lds, st>>>(sys, rec, pass, xcd); break;
    case K_R2C: batch_fft_kernel<T, K_R2C, OFF><<<grid, block, lds, st>>>(sys, rec, pass, xcd); break;
    case K_C2R: batch_fft_kernel<T, K_C2R, OFF><<<grid, block, lds, st>>>(sys, rec, pass, xcd); break;
    default: batch_fft_kernel<T, K_FUSED, OFF><<<grid, block, lds, st>>>(sys, rec, pass, xcd); break;
  }
}

void launch_batch_fft(bool f64, int kind, bool wide, const SysDesc* sys, const int4* rec, int pass, int nitems,
                      size_t lds, int xcd, hipStream_t st) {
  if (nitems <= 0) return;
  using W = unsigned long long;
  if (f64) wide ? launch_batch_fft_t<double, W>(kind, sys, rec, pass, nitems, lds, xcd, st)
                : launch_batch_fft_t<double, unsigned>(kind, sys, rec, pass, nitems, lds, xcd, st);
  else wide ? launch_batch_fft_t<float, W>(kind, sys, rec, pass, nitems, lds, xcd, st)
            : launch_batch_fft_t<float, unsigned>(kind, sys, rec, pass, nitems, lds, xcd, st);
}

}  // namespace se
