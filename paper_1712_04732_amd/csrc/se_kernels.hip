// gfx950 kernels of the Spectral Ewald k-space path (Algorithm 4 of
// Shamshirgar, Bagge, Tornberg, arXiv:1712.04732).
//
//   bin      : grid cell, fractional offset and tile of every particle; tile
//              counting sort (implementation of the gridding loop bounds).
//   spread   : Eq. (gridding).  Output-stationary: one workgroup owns one tile
//              of the grid, accumulates every particle whose P^3 stencil meets
//              the tile into an LDS copy of the tile, and writes the tile once.
//              No global atomics; grid bytes are written exactly once.
//   fft      : pencil transforms, in se_fft.hip.
//   gather   : trapezoidal rule of Eq. (complete_integral) and its gradient,
//              Eq. (force-method-1).  One workgroup per tile stages the
//              tile's stencil region of the grid in LDS; one wavefront per
//              particle, 64 lanes over the stencil columns, cross-lane
//              reduction by shuffles.
//   energy   : FP64 reduction of q phi.
//   0P       : Algorithm 3 helpers in FP64.
#include "se_device.h"

namespace se {

// A coordinate of direction d folded into the grid: periodic directions wrap
// (any number of periods), free directions report points outside [0, G).
__device__ __forceinline__ int wrap_coord(const GridGeom& g, int d, int c, bool* ok) {
  const int G = g.G[d];
  if (g.per[d]) {
    c %= G;
    return c < 0 ? c + G : c;
  }
  *ok = *ok && c >= 0 && c < G;
  return c;
}


// ---------------------------------------------------------------------------
// Binning: grid cell, fractional offset and sub-bin of every particle.  The
// sub-bins are blocks of kSB^3 cells; sorting the particles by sub-bin lets a
// tile find every particle whose stencil can reach it as a short list of
// contiguous index ranges.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pack_cell(int cx_, int cy, int cz) { return cx_ | (cy << 10) | (cz << 20); }

template <typename T>
__device__ __forceinline__ T warp_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Sum over aligned groups of W lanes (W a power of two <= 64).
template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int m = W / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// LDS writes of a wavefront made visible to the other lanes of the same wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int sb_key(const GridGeom& g, int cx_, int cy, int cz) {
  return ((cz / kSB) * g.nsb[1] + cy / kSB) * g.nsb[0] + cx_ / kSB;
}

template <typename Tin, typename T>
__device__ __forceinline__ void stage_bin(const GridGeom& g, const EvalBuffers& b, long N, const Tin* __restrict__ xyz,
                          const Tin* __restrict__ q, int item) {
  const long n = (long)item * blockDim.x + threadIdx.x;
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
        const double Ld = g.Lp[d];
        const double xw = x - Ld * floor(x / Ld);
        t = xw / g.h;
        ci = (int)floor(t);
        if (ci >= g.G[d] || ci < 0) {  // xw rounded up to L
          ci = 0;
          t = 0.0;
        }
      } else {
        if (!(x >= 0.0 && x < g.L)) bad |= 2;
        t = x / g.h + g.d0[d];
        ci = (int)floor(t);
        const int lo = g.d0[d], hi = g.G[d] - g.d0[d] - 1;
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
    const int key = sb_key(g, c[0], c[1], c[2]);
    b.p_key[n] = key;
    b.p_cell[n] = pack_cell(c[0], c[1], c[2]);
    reinterpret_cast<Quad<T>*>(b.p_frac)[n] = Quad<T>{(T)f[0], (T)f[1], (T)f[2], (T)qn};
    atomicAdd(&b.sb_count[key], 1);
    sq = qn;
    sa = fabs(qn);
    s2 = qn * qn;
  }
  // block partial sums of the charges (FP64), for the neutrality check and Q,
  // and the block's largest |q| (bounds the spreading's fixed-point range)
  __shared__ double red[4][kBlock / 64];
  double smax = sa;
  sq = warp_sum(sq);
  sa = warp_sum(sa);
  s2 = warp_sum(s2);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) smax = fmax(smax, __shfl_xor(smax, m, 64));
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) {
    red[0][w] = sq;
    red[1][w] = sa;
    red[2][w] = s2;
    red[3][w] = smax;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int i = 0; i < kBlock / 64; ++i)
      s = threadIdx.x == 3 ? fmax(s, red[3][i]) : s + red[threadIdx.x][i];
    b.qpart[4 * item + threadIdx.x] = s;
  }
}

template <typename Tin, typename T>
__global__ __launch_bounds__(kBlock) void bin_kernel(GridGeom g, EvalBuffers b, long N,
                                                     const Tin* __restrict__ xyz,
                                                     const Tin* __restrict__ q) {
  stage_bin<Tin, T>(g, b, N, xyz, q, blockIdx.x);
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

// Exclusive scan of the sub-bin counts in two passes over blocks of
// kScanBlock entries: a local scan with block totals, then each block adds the
// sum of the totals before it.  Block 0 of the second pass also reduces the
// FP64 charge sums and applies the neutrality check.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ void stage_scan1(const GridGeom& g, const EvalBuffers& b, int item) {
  const int n = g.nsb[0] * g.nsb[1] * g.nsb[2];
  const int base = item * kScanBlock;
  constexpr int K = kScanBlock / kBlock;
  int v[K];
  int s = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = base + threadIdx.x * K + k;
    v[k] = i < n ? b.sb_count[i] : 0;
    s += v[k];
  }
  __shared__ int part[kBlock];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = base + threadIdx.x * K + k;
    if (i < n) b.sb_start[i] = run;
    run += v[k];
  }
  if (threadIdx.x == kBlock - 1) b.bsum[item] = part[kBlock - 1];
}

__global__ __launch_bounds__(kBlock) void scan1_kernel(GridGeom g, EvalBuffers b) {
  stage_scan1(g, b, blockIdx.x);
}

__device__ __forceinline__ void stage_scan2(const GridGeom& g, const EvalBuffers& b, int nblk_bin, int check_neutral,
                            int item, int nscan) {
  const int n = g.nsb[0] * g.nsb[1] * g.nsb[2];
  __shared__ int ps[kBlock];
  __shared__ double dq[4][kBlock];
  int o = 0;
  for (int j = threadIdx.x; j < item; j += kBlock) o += b.bsum[j];
  ps[threadIdx.x] = o;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) ps[threadIdx.x] += ps[threadIdx.x + off];
    __syncthreads();
  }
  const int offset = ps[0];
  const int base = item * kScanBlock;
  for (int k = threadIdx.x; k < kScanBlock; k += kBlock) {
    const int i = base + k;
    if (i < n) {
      const int v = b.sb_start[i] + offset;
      b.sb_start[i] = v;
      b.sb_cursor[i] = v;
    }
  }
  if (item == nscan - 1 && threadIdx.x == 0) b.sb_start[n] = offset + b.bsum[item];
  if (item != 0) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int i = threadIdx.x; i < nblk_bin; i += kBlock) {
    a0 += b.qpart[4 * i];
    a1 += b.qpart[4 * i + 1];
    a2 += b.qpart[4 * i + 2];
    a3 = fmax(a3, b.qpart[4 * i + 3]);
  }
  dq[0][threadIdx.x] = a0;
  dq[1][threadIdx.x] = a1;
  dq[2][threadIdx.x] = a2;
  dq[3][threadIdx.x] = a3;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      dq[0][threadIdx.x] += dq[0][threadIdx.x + off];
      dq[1][threadIdx.x] += dq[1][threadIdx.x + off];
      dq[2][threadIdx.x] += dq[2][threadIdx.x + off];
      dq[3][threadIdx.x] = fmax(dq[3][threadIdx.x], dq[3][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    b.red[0] = dq[0][0];
    b.red[1] = dq[1][0];
    b.red[2] = dq[2][0];
    b.red[3] = dq[3][0];
    if (check_neutral && fabs(dq[0][0]) > 1e-10 * dq[1][0]) atomicOr(b.status, 4);
  }
}

__global__ __launch_bounds__(kBlock) void scan2_kernel(GridGeom g, EvalBuffers b, int nblk_bin,
                                                       int check_neutral) {
  stage_scan2(g, b, nblk_bin, check_neutral, blockIdx.x, gridDim.x);
}

int scan_blocks(const GridGeom& g) {
  return (g.nsb[0] * g.nsb[1] * g.nsb[2] + kScanBlock - 1) / kScanBlock;
}

hipError_t launch_scan(const GridGeom& g, const EvalBuffers& b, int nblk_bin, int check_neutral,
                       hipStream_t st) {
  const int nb = scan_blocks(g);
  scan1_kernel<<<dim3(nb), dim3(kBlock), 0, st>>>(g, b);
  scan2_kernel<<<dim3(nb), dim3(kBlock), 0, st>>>(g, b, nblk_bin, check_neutral);
  return hipGetLastError();
}

template <typename T>
__device__ __forceinline__ void stage_scatter(const EvalBuffers& b, long N, int item) {
  const long n = (long)item * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int key = b.p_key[n];
  const int pos = atomicAdd(&b.sb_cursor[key], 1);
  b.s_cell[pos] = b.p_cell[n];
  b.s_idx[pos] = (int)n;
  reinterpret_cast<Quad<T>*>(b.s_fq)[pos] = reinterpret_cast<const Quad<T>*>(b.p_frac)[n];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scatter_kernel(EvalBuffers b, long N) {
  stage_scatter<T>(b, N, blockIdx.x);
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

// Order each sub-bin's particles by input index.  The scatter fills a
// sub-bin's slots in the order its atomic cursor is taken, which varies
// between runs; spreading modes that sum in floating point in particle order
// need a fixed order to give the same result every time.  One thread per
// sub-bin, insertion sort of its (short) segment in place.
template <typename T>
__device__ __forceinline__ void stage_order(const EvalBuffers& b, int nsbtot, int item) {
  const int k = item * blockDim.x + threadIdx.x;
  if (k >= nsbtot) return;
  const int a = b.sb_start[k], e = b.sb_start[k + 1];
  Quad<T>* fq = reinterpret_cast<Quad<T>*>(b.s_fq);
  for (int j = a + 1; j < e; ++j) {
    const int idx = b.s_idx[j];
    if (b.s_idx[j - 1] <= idx) continue;
    const int cell = b.s_cell[j];
    const Quad<T> f = fq[j];
    int i = j - 1;
    while (i >= a && b.s_idx[i] > idx) {
      b.s_idx[i + 1] = b.s_idx[i];
      b.s_cell[i + 1] = b.s_cell[i];
      fq[i + 1] = fq[i];
      --i;
    }
    b.s_idx[i + 1] = idx;
    b.s_cell[i + 1] = cell;
    fq[i + 1] = f;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void order_kernel(EvalBuffers b, int nsbtot) {
  stage_order<T>(b, nsbtot, blockIdx.x);
}

hipError_t launch_order(const GridGeom& g, const EvalBuffers& b, int nsbtot, bool f64, hipStream_t st) {
  (void)g;
  const dim3 grid((unsigned)((nsbtot + kBlock - 1) / kBlock)), block(kBlock);
  if (f64)
    order_kernel<double><<<grid, block, 0, st>>>(b, nsbtot);
  else
    order_kernel<float><<<grid, block, 0, st>>>(b, nsbtot);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window weights (Section 4).  f = frac(t) of the particle's grid coordinate,
// stencil point i at grid index floor(t) - P/2 + 1 + i.
//   PKB: xbar = 1 - 2f for all i (Section 4.1), Horner on row i of the
//        coefficient table; the derivative table already carries d/dx
//        (chain factor -2/h).
//   Gaussian: u = i + 1 - P/2 - f (grid units), W = exp(-alpha (2u/P)^2),
//        dW/dx = W 2 alpha (2/P)^2 u / h.
//   ES: W = exp(beta (sqrt(1 - z^2) - 1)), z = 2u/P (beta held in alpha).
// ---------------------------------------------------------------------------
// Segments are {first0, last0, first1, last1} in sub-bin units.
__device__ __forceinline__ int seg_len(const int* seg, int ns) {
  int n = 0;
  for (int k = 0; k < ns; ++k) n += seg[2 * k + 1] - seg[2 * k] + 1;
  return n;
}

__device__ __forceinline__ int seg_at(const int* seg, int ns, int r) {
  const int l0 = seg[1] - seg[0] + 1;
  return (ns == 1 || r < l0) ? seg[0] + r : seg[2] + (r - l0);
}

__device__ int prefix_ranges(int* rpre, int nr);

// Particle index ranges of the sub-bin rows (z, y, x-segment) of a tile's
// anchor box, and their exclusive prefix; returns the total particle count.
// All threads of the block call it; ends with a barrier.
__device__ int build_ranges(const GridGeom& g, const EvalBuffers& b, const int* sz, int nsz,
                            const int* sy, int nsy, const int* sx, int nsx, int* rstart, int* rpre) {
  const int nz = seg_len(sz, nsz), ny = seg_len(sy, nsy);
  const int nr = nz * ny * nsx;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    const int xs = r % nsx, ry = (r / nsx) % ny, rz = r / (nsx * ny);
    const int bz = seg_at(sz, nsz, rz), by = seg_at(sy, nsy, ry);
    const int row = (bz * g.nsb[1] + by) * g.nsb[0];
    const auto sbs = gld(b.sb_start);
    const int a = sbs[row + sx[2 * xs]], e = sbs[row + sx[2 * xs + 1] + 1];
    rstart[r] = a;
    rpre[r] = e - a;
  }
  __syncthreads();
  return prefix_ranges(rpre, nr);
}

// Exclusive prefix of rpre[0..nr) in place, rpre[nr] = total; returns the
// total.  All threads of the block call it; ends with a barrier.  Up to 64
// ranges (every tile of side <= 32 at kSB = 4) one wavefront scans them by
// lane shuffles, so the block waits at one barrier instead of two per
// doubling step.
__device__ int prefix_ranges(int* rpre, int nr) {
  if (nr <= 64) {
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      const int c = lane < nr ? rpre[lane] : 0;
      int v = c;   // inclusive prefix; lanes at and past nr add 0, so lane 63 holds the total
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int w = __shfl_up(v, o, 64);
        if (lane >= o) v += w;
      }
      if (lane < nr) rpre[lane] = v - c;
      if (lane == 63) rpre[nr] = v;
    }
    __syncthreads();
    return rpre[nr];
  }
  __shared__ int part[kMaxBlock];
  const int per = (nr + blockDim.x - 1) / blockDim.x;
  const int lo = min(nr, (int)threadIdx.x * per), hi = min(nr, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += rpre[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int i = lo; i < hi; ++i) {
    const int c = rpre[i];
    rpre[i] = run;
    run += c;
  }
  const int total = part[blockDim.x - 1];
  __syncthreads();
  if (threadIdx.x == 0) rpre[nr] = total;
  __syncthreads();
  return total;
}

// Range holding flattened index e: the last r with rpre[r] <= e.
__device__ __forceinline__ int find_range(const int* rpre, int nr, int e) {
  int lo = 0, hi = nr - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rpre[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Spreading, Eq. (gridding), in two kernels.
//   spread: one workgroup per tile takes the particles anchored in the tile
//     and adds their full P^3 stencils into an LDS box covering the tile and
//     its stencil halo, (T+P-1)^3 points; each wavefront evaluates the weights
//     of 64 particles at a time (one lane per particle), then adds them one
//     particle at a time, 64 lanes over the stencil columns (ix, iy) and a loop
//     over iz; the box is stored once to a staging array.
//   fold: one workgroup per tile sums, for each of its grid points, the boxes
//     of the up to 27 tiles (periodic images included) that cover the point,
//     in a fixed order, and writes the grid point once.
// No global atomics.
// ---------------------------------------------------------------------------
// Lanes per particle when one lane evaluates one row of the window weights.
template <int P>
struct Lanes {
  static constexpr int G2 = P <= 2 ? 2 : (P <= 4 ? 4 : (P <= 8 ? 8 : 16));
  static constexpr int PPW = 64 / G2;
};

// Gathering serves one particle with P lanes (one per stencil plane), so a
// wavefront takes floor(64 / P) particles; a power-of-two group would leave
// next_pow2(P) - P lanes of every group idle (6 of 16 at P = 10).  FP64
// takes at most 4 particles per wavefront, which keeps the weight rows of
// 8^3 tiles within the LDS budget.
template <int P, typename T>
struct GatherLanes {
  static constexpr int G = P < 2 ? 2 : P;
  static constexpr int PPW = sizeof(T) == 8 && 64 / G > 4 ? 4 : 64 / G;
};

// Sum over the G consecutive lanes of a group (lane iz of the group); the
// result is complete at iz = 0.  Step o adds lane iz + o, which holds the
// sum of lanes iz + o .. iz + 2o - 1 of the group, when it lies in the group.
template <int G, typename T>
__device__ __forceinline__ T segment_sum(T v, int iz) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
    const T w = __shfl_down(v, o, 64);
    if (iz + o < G) v += w;
  }
  return v;
}

// Row i of the PKB coefficient table (values or derivatives) in registers.
template <typename T>
__device__ __forceinline__ void load_row(const T* __restrict__ tab, int i, int m, T* r) {
  const auto t = gld(tab);
#pragma unroll
  for (int j = 0; j <= kMaxNu; ++j) r[j] = j < m ? t[i * m + j] : (T)0;
}

// Window weight of stencil row i at fractional offset f from a register row.
template <typename T, int P>
__device__ __forceinline__ T weight_reg(const GridGeom& g, const T* r, int i, T f) {
  if (g.window == 1) {
    const T xb = (T)1 - (T)2 * f;
    T a = r[kMaxNu];
#pragma unroll
    for (int j = kMaxNu - 1; j >= 0; --j) a = a * xb + r[j];
    return a;
  }
  const T u = (T)(i + 1 - P / 2) - f;
  if (g.window == 2) {
    // ES window, Eq. (expsemicirc_window): e^{beta (sqrt(1 - z^2) - 1)}, z = 2u/P
    const T z = (T)2 * u / (T)P;
    return exp((T)g.alpha * (sqrt(max((T)1 - z * z, (T)0)) - (T)1));
  }
  return exp(-(T)g.alpha * ((T)4 / (T)(P * P)) * u * u);
}

template <typename T, int P>
__device__ __forceinline__ T dweight_reg(const GridGeom& g, const T* r, int i, T f) {
  if (g.window == 1) return weight_reg<T, P>(g, r, i, f);
  const T u = (T)(i + 1 - P / 2) - f;
  if (g.window == 2) {
    // d/dx of the ES window at u = grid point - particle: W beta z (2/P) / sqrt(1 - z^2) / h,
    // 0 at the end points (not differentiable there)
    const T z = (T)2 * u / (T)P, s2 = (T)1 - z * z;
    if (!(s2 > (T)0)) return (T)0;
    const T s = sqrt(s2);
    return exp((T)g.alpha * (s - (T)1)) * (T)g.alpha * z * ((T)2 / (T)P) / (s * (T)g.h);
  }
  const T c2 = (T)4 / (T)(P * P);
  return exp(-(T)g.alpha * c2 * u * u) * (T)2 * (T)g.alpha * c2 * u / (T)g.h;
}

// Round d to the nearest integer for |d| < 2^51: adding 1.5 * 2^52 moves the
// integer part into the low mantissa bits.
__device__ __forceinline__ long long round_fixed(double d) {
  return __double_as_longlong(d + 6755399441055744.0) - 0x4338000000000000LL;
}

template <typename T, int P>
__device__ __forceinline__ void stage_spread(const GridGeom& g, const EvalBuffers& b, int item, unsigned char* smem) {
  constexpr int G2 = Lanes<P>::G2, PPW = Lanes<P>::PPW;
  const int TX = g.T[0], TY = g.T[1], TZ = g.T[2];
  const int t_id = item;
  const int tz = t_id / (g.nt[0] * g.nt[1]);
  const int ty = (t_id / g.nt[0]) % g.nt[1];
  const int tx = t_id % g.nt[0];
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int ex = min(TX, g.G[0] - x0), ey = min(TY, g.G[1] - y0), ez = min(TZ, g.G[2] - z0);
  const int RX = TX + P - 1, RY = TY + P - 1, RZ = TZ + P - 1, R3 = RX * RY * RZ;
  const int m = g.nu + 1;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nwaves = blockDim.x / 64;
  const int CH = g.chunk;                                     // particles per wavefront round

  unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem);   // R3, fixed point
  int* rstart = reinterpret_cast<int*>(acc + R3);             // kMaxOwnRanges
  int* rpre = rstart + kMaxOwnRanges;                         // kMaxOwnRanges + 1
  T* wbuf = reinterpret_cast<T*>(rpre + kMaxOwnRanges + 4);   // nwaves * CH * 3P
  int* obuf = reinterpret_cast<int*>(wbuf + nwaves * CH * 3 * P);  // nwaves * CH * 3
  Quad<T>* rbuf = reinterpret_cast<Quad<T>*>(obuf + nwaves * CH * 3 + 4);  // nwaves * CH

  for (int i = threadIdx.x; i < R3; i += blockDim.x) acc[i] = 0ull;
  int sx[2] = {x0 / kSB, (x0 + ex - 1) / kSB}, sy[2] = {y0 / kSB, (y0 + ey - 1) / kSB},
      sz[2] = {z0 / kSB, (z0 + ez - 1) / kSB};
  const int nr = (sz[1] - sz[0] + 1) * (sy[1] - sy[0] + 1);
  const int total = build_ranges(g, b, sz, 1, sy, 1, sx, 1, rstart, rpre);

  // Fixed-point scale of this tile: |sum of q W| at any point is at most
  // (particles) x max |q| (W <= 1), kept below 2^50.
  const double stile = (double)total * gld(b.red)[3];
  const double scale = stile > 0.0 ? 1125899906842624.0 / (1.0009765625 * stile) : 0.0;   // 2^50

  // coefficient row of this lane (row k = lane % G2)
  const int kr = lane % G2, pr = lane / G2;
  T crow[kMaxNu + 1];
  load_row(reinterpret_cast<const T*>(b.wtab), min(kr, P - 1), m, crow);

  T* ww = wbuf + wave * CH * 3 * P;
  int* wo = obuf + wave * CH * 3;
  Quad<T>* wr = rbuf + wave * CH;
  const int RXY = RX * RY;
  for (int base = wave * CH; base < total; base += nwaves * CH) {
    const int nv = min(CH, total - base);
    // the chunk's particle records, one per lane in one round of loads
    if (lane < nv) {
      const int e = base + lane;
      const int r = find_range(rpre, nr, e);
      const int i = rstart[r] + (e - rpre[r]);
      wr[lane] = ld_quad<T>(b.s_fq, i);
      const int pc = gld(b.s_cell)[i];
      // stencil origin c - P/2 + 1 in box coordinates (box origin x0 - P/2 + 1)
      wo[3 * lane] = (pc & 1023) - x0;
      wo[3 * lane + 1] = ((pc >> 10) & 1023) - y0;
      wo[3 * lane + 2] = ((pc >> 20) & 1023) - z0;
    }
    wave_sync();
    // weights: G2 lanes per particle, lane k evaluates row k in x, y, z
    for (int p0 = 0; p0 < nv; p0 += PPW) {
      const int p = p0 + pr;
      if (p < nv && kr < P) {
        const Quad<T> f = wr[p];
        T* w = ww + p * 3 * P;
        w[kr] = weight_reg<T, P>(g, crow, kr, f.fx);
        w[P + kr] = weight_reg<T, P>(g, crow, kr, f.fy);
        w[2 * P + kr] = f.q * weight_reg<T, P>(g, crow, kr, f.fz);
      }
    }
    wave_sync();
    for (int s = 0; s < nv; ++s) {
      const int ox = wo[3 * s], oy = wo[3 * s + 1], oz = wo[3 * s + 2];
      const T* w = ww + s * 3 * P;
      T wz[P];
#pragma unroll
      for (int k = 0; k < P; ++k) wz[k] = w[2 * P + k];
      for (int l = lane; l < P * P; l += 64) {
        const int ix = l % P, iy = l / P;
        const double wxy = (double)(w[ix] * w[P + iy]) * scale;
        unsigned long long* col = acc + (oz * RY + oy + iy) * RX + ox + ix;
#pragma unroll
        for (int iz = 0; iz < P; ++iz)
          atomicAdd(col + iz * RXY, (unsigned long long)round_fixed(wxy * (double)wz[iz]));
      }
    }
    wave_sync();
  }
  __syncthreads();
  T* stg = reinterpret_cast<T*>(b.stage) + (long long)t_id * R3;
  const double inv = stile > 0.0 ? 1.0 / scale : 0.0;
  for (int i = threadIdx.x; i < R3; i += blockDim.x) gst(stg)[i] = (T)((double)(long long)acc[i] * inv);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Spreading straight into the grid (no staging, no fold).  One workgroup per
// tile takes every particle whose stencil reaches the tile -- its own and its
// neighbours', periodic images included -- and adds the part of each stencil
// that falls inside the tile into an LDS copy of the tile alone (T^3 points,
// 64-bit fixed point as above), then writes the tile once.  A particle near a
// tile boundary is visited by every tile its stencil reaches; the stencil
// points it adds are split among those tiles.  Suited to sparse grids, where
// staging (T+P-1)^3 boxes costs more than the particles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((b - 1 - a) / b); }

// Anchor cells [lo, hi] (unwrapped) of one direction as pieces of the grid:
// sub-bin segment [s0, s1] and the image shift added to the cells of the
// piece.  Returns the number of pieces (at most kMaxPieces; the planner
// rejects geometries needing more).
__device__ __forceinline__ int anchor_pieces(const GridGeom& g, int d, int lo, int hi, int* s0, int* s1,
                                             int* shift) {
  const int G = g.G[d];
  int n = 0;
  if (!g.per[d]) {
    lo = max(lo, 0);
    hi = min(hi, G - 1);
    if (lo <= hi) {
      s0[0] = lo / kSB;
      s1[0] = hi / kSB;
      shift[0] = 0;
      n = 1;
    }
    return n;
  }
  for (int k = floor_div(lo, G); k <= floor_div(hi, G) && n < kMaxPieces; ++k) {
    const int a = max(lo - k * G, 0), e = min(hi - k * G, G - 1);
    if (a > e) continue;
    s0[n] = a / kSB;
    s1[n] = e / kSB;
    shift[n] = k * G;
    ++n;
  }
  return n;
}

template <typename T, int P>
__device__ __forceinline__ void stage_spread_clip(const GridGeom& g, const EvalBuffers& b, int item,
                                                  unsigned char* smem) {
  constexpr int G2 = Lanes<P>::G2, PPW = Lanes<P>::PPW;
  const int TX = g.T[0], TY = g.T[1], TZ = g.T[2];
  const int tz = item / (g.nt[0] * g.nt[1]);
  const int ty = (item / g.nt[0]) % g.nt[1];
  const int tx = item % g.nt[0];
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int ex = min(TX, g.G[0] - x0), ey = min(TY, g.G[1] - y0), ez = min(TZ, g.G[2] - z0);
  const int T3 = TX * TY * TZ, TXY = TX * TY;
  const int m = g.nu + 1;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nwaves = blockDim.x / 64;
  const int CH = g.chunk;

  unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem);   // T3, fixed point
  int* rstart = reinterpret_cast<int*>(acc + T3);             // kMaxClipRanges
  int* rpre = rstart + kMaxClipRanges;                        // kMaxClipRanges + 1
  int* rsh = rpre + kMaxClipRanges + 4;                       // kMaxClipRanges
  T* wbuf = reinterpret_cast<T*>(rsh + kMaxClipRanges);       // nwaves * CH * 3P
  int* obuf = reinterpret_cast<int*>(wbuf + nwaves * CH * 3 * P);  // nwaves * CH * 3
  Quad<T>* rbuf = reinterpret_cast<Quad<T>*>(obuf + nwaves * CH * 3 + 4);  // nwaves * CH
  __shared__ int pc_s0[3][kMaxPieces], pc_s1[3][kMaxPieces], pc_sh[3][kMaxPieces], pc_n[3];

  for (int i = threadIdx.x; i < T3; i += blockDim.x) acc[i] = 0ull;
  if (threadIdx.x < 3) {
    const int d = threadIdx.x, o = d == 0 ? x0 : (d == 1 ? y0 : z0), e = d == 0 ? ex : (d == 1 ? ey : ez);
    // anchors c whose stencil c - P/2 + 1 .. c + P/2 meets [o, o + e)
    pc_n[d] = anchor_pieces(g, d, o - P / 2, o + e - 1 + P / 2 - 1, pc_s0[d], pc_s1[d], pc_sh[d]);
  }
  __syncthreads();
  // ranges: (z piece, z sub-bin) x (y piece, y sub-bin) x x piece
  int nzb = 0, nyb = 0;
  for (int k = 0; k < pc_n[2]; ++k) nzb += pc_s1[2][k] - pc_s0[2][k] + 1;
  for (int k = 0; k < pc_n[1]; ++k) nyb += pc_s1[1][k] - pc_s0[1][k] + 1;
  const int npx = pc_n[0];
  const int nr = nzb * nyb * npx;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    const int xs = r % npx, ry = (r / npx) % nyb, rz = r / (npx * nyb);
    int kz = 0, bz = rz, ky = 0, by = ry;
    while (bz > pc_s1[2][kz] - pc_s0[2][kz]) bz -= pc_s1[2][kz] - pc_s0[2][kz] + 1, ++kz;
    while (by > pc_s1[1][ky] - pc_s0[1][ky]) by -= pc_s1[1][ky] - pc_s0[1][ky] + 1, ++ky;
    bz += pc_s0[2][kz];
    by += pc_s0[1][ky];
    const int row = (bz * g.nsb[1] + by) * g.nsb[0];
    const auto sbs = gld(b.sb_start);
    const int a = sbs[row + pc_s0[0][xs]], e = sbs[row + pc_s1[0][xs] + 1];
    rstart[r] = a;
    rpre[r] = e - a;
    rsh[r] = kz | (ky << 4) | (xs << 8);
  }
  __syncthreads();
  const int total = prefix_ranges(rpre, nr);

  // fixed-point scale: every tile point is bounded by (visits) x max |q|
  const double stile = (double)total * gld(b.red)[3];
  const double scale = stile > 0.0 ? 1125899906842624.0 / (1.0009765625 * stile) : 0.0;   // 2^50

  const int kr = lane % G2, pr = lane / G2;
  T crow[kMaxNu + 1];
  load_row(reinterpret_cast<const T*>(b.wtab), min(kr, P - 1), m, crow);

  T* ww = wbuf + wave * CH * 3 * P;
  int* wo = obuf + wave * CH * 3;
  Quad<T>* wr = rbuf + wave * CH;
  for (int base = wave * CH; base < total; base += nwaves * CH) {
    const int nv = min(CH, total - base);
    // the chunk's particle records, one per lane in one round of loads
    if (lane < nv) {
      const int e = base + lane;
      const int r = find_range(rpre, nr, e);
      const int i = rstart[r] + (e - rpre[r]);
      wr[lane] = ld_quad<T>(b.s_fq, i);
      const int pc = gld(b.s_cell)[i], code = rsh[r];
      // stencil origin c + shift - P/2 + 1 in tile coordinates
      wo[3 * lane] = (pc & 1023) + pc_sh[0][code >> 8] - P / 2 + 1 - x0;
      wo[3 * lane + 1] = ((pc >> 10) & 1023) + pc_sh[1][(code >> 4) & 15] - P / 2 + 1 - y0;
      wo[3 * lane + 2] = ((pc >> 20) & 1023) + pc_sh[2][code & 15] - P / 2 + 1 - z0;
    }
    wave_sync();
    for (int p0 = 0; p0 < nv; p0 += PPW) {
      const int p = p0 + pr;
      if (p < nv && kr < P) {
        const Quad<T> f = wr[p];
        T* w = ww + p * 3 * P;
        w[kr] = weight_reg<T, P>(g, crow, kr, f.fx);
        w[P + kr] = weight_reg<T, P>(g, crow, kr, f.fy);
        w[2 * P + kr] = f.q * weight_reg<T, P>(g, crow, kr, f.fz);
      }
    }
    wave_sync();
    for (int s = 0; s < nv; ++s) {
      const int ox = wo[3 * s], oy = wo[3 * s + 1], oz = wo[3 * s + 2];
      const T* w = ww + s * 3 * P;
      T wz[P];
#pragma unroll
      for (int k = 0; k < P; ++k) wz[k] = w[2 * P + k];
      // the stencil's z overlap with the tile is the same for all lanes
      const int iz0 = max(0, -oz), iz1 = min(P, ez - oz);
      for (int l = lane; l < P * P; l += 64) {
        const int lx = ox + l % P, ly = oy + l / P;
        if ((unsigned)lx >= (unsigned)ex || (unsigned)ly >= (unsigned)ey) continue;
        const double wxy = (double)(w[l % P] * w[P + l / P]) * scale;
        unsigned long long* col = acc + ly * TX + lx;
#pragma unroll
        for (int iz = 0; iz < P; ++iz)
          if (iz >= iz0 && iz < iz1)
            atomicAdd(col + (oz + iz) * TXY, (unsigned long long)round_fixed(wxy * (double)wz[iz]));
      }
    }
    wave_sync();
  }
  __syncthreads();
  T* grid = reinterpret_cast<T*>(b.grid);
  const double inv = stile > 0.0 ? 1.0 / scale : 0.0;
  {
    // rows of the tile, 64 / TX rows per wavefront at a time
    const int rpw = 64 / TX, sub = lane / TX, lx = lane - sub * TX;
    const int nrows = ey * ez;
    if (sub < rpw && lx < ex)
      for (int r0 = wave * rpw; r0 < nrows; r0 += nwaves * rpw) {
        const int row = r0 + sub;
        if (row >= nrows) break;
        const int ly = row % ey, lz = row / ey;
        gst(grid)[((long long)(z0 + lz) * g.G[1] + y0 + ly) * g.G[0] + x0 + lx] =
            (T)((double)(long long)acc[(lz * TY + ly) * TX + lx] * inv);
      }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Spreading by columns (no atomics, no staging, no fold).  One workgroup per
// tile.  The particles whose stencils reach the tile (periodic images
// included, as for the clipped mode) are taken in batches: each thread
// evaluates the 3P window weights of one particle into LDS.  Each thread then
// owns two neighbouring grid columns (x0 + 2i, x0 + 2i + 1; y) and keeps their
// TZ values in registers; the two halves of the workgroup take the even and
// the odd visits of a batch, and add their sums at the end in a fixed order.
// A visit's x weights sit in a row padded with a zero on each side, so both
// columns of a thread read their weight without a range test; the z weights
// are a whole row in the tile's z frame (zeros outside the stencil), so every
// visit adds 2 x kColZ products to fixed registers.  Sums run in the compute
// precision in a fixed particle order.
// ---------------------------------------------------------------------------
template <typename T, int P>
struct ColLayout {
  // per visit: the z row (kColZ), the zero-padded x row (P + 2), the y row (P);
  // records 16-byte aligned
  static constexpr int XO = kColZ, YO = kColZ + P + 2;
  static constexpr int SW = (YO + P + 3) / 4 * 4;
};

template <typename T, int P>
__device__ __forceinline__ void stage_spread_cols(const GridGeom& g, const EvalBuffers& b, int item,
                                                  unsigned char* smem) {
  using Lay = ColLayout<T, P>;
  constexpr int SW = Lay::SW, XO = Lay::XO, YO = Lay::YO;
  const int TX = g.T[0], TY = g.T[1], TZ = g.T[2];
  const int tz = item / (g.nt[0] * g.nt[1]);
  const int ty = (item / g.nt[0]) % g.nt[1];
  const int tx = item % g.nt[0];
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int ex = min(TX, g.G[0] - x0), ey = min(TY, g.G[1] - y0), ez = min(TZ, g.G[2] - z0);
  const int m = g.nu + 1;

  int* rstart = reinterpret_cast<int*>(smem);                 // kMaxClipRanges
  int* rpre = rstart + kMaxClipRanges;                        // kMaxClipRanges + 1
  int* rsh = rpre + kMaxClipRanges + 4;                       // kMaxClipRanges
  int* org = rsh + kMaxClipRanges;                            // kColBatch packed origins
  T* wb = reinterpret_cast<T*>(org + kColBatch);              // kColBatch records of SW weights
  constexpr int WBN = kColBatch * SW > kBlock * kColZ ? kColBatch * SW : kBlock * kColZ;
  Quad<T>* pq = reinterpret_cast<Quad<T>*>(wb + WBN);          // kColBatch particle records
  int* ppc = reinterpret_cast<int*>(pq + kColBatch);           // their packed cells
  int* pcd = ppc + kColBatch;                                  // and image-shift codes
  __shared__ int pc_s0[3][kMaxPieces], pc_s1[3][kMaxPieces], pc_sh[3][kMaxPieces], pc_n[3];

  if (threadIdx.x < 3) {
    const int d = threadIdx.x, o = d == 0 ? x0 : (d == 1 ? y0 : z0), e = d == 0 ? ex : (d == 1 ? ey : ez);
    pc_n[d] = anchor_pieces(g, d, o - P / 2, o + e - 1 + P / 2 - 1, pc_s0[d], pc_s1[d], pc_sh[d]);
  }
  __syncthreads();
  int nzb = 0, nyb = 0;
  for (int k = 0; k < pc_n[2]; ++k) nzb += pc_s1[2][k] - pc_s0[2][k] + 1;
  for (int k = 0; k < pc_n[1]; ++k) nyb += pc_s1[1][k] - pc_s0[1][k] + 1;
  const int npx = pc_n[0];
  const int nr = nzb * nyb * npx;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    const int xs = r % npx, ry = (r / npx) % nyb, rz = r / (npx * nyb);
    int kz = 0, bz = rz, ky = 0, by = ry;
    while (bz > pc_s1[2][kz] - pc_s0[2][kz]) bz -= pc_s1[2][kz] - pc_s0[2][kz] + 1, ++kz;
    while (by > pc_s1[1][ky] - pc_s0[1][ky]) by -= pc_s1[1][ky] - pc_s0[1][ky] + 1, ++ky;
    bz += pc_s0[2][kz];
    by += pc_s0[1][ky];
    const int row = (bz * g.nsb[1] + by) * g.nsb[0];
    const auto sbs = gld(b.sb_start);
    const int a = sbs[row + pc_s0[0][xs]], e = sbs[row + pc_s1[0][xs] + 1];
    rstart[r] = a;
    rpre[r] = e - a;
    rsh[r] = kz | (ky << 4) | (xs << 8);
  }
  __syncthreads();
  const int total = prefix_ranges(rpre, nr);

  // column pair and visit parity of this thread (the parity is wavefront-uniform)
  const int half = (int)threadIdx.x >= kBlock / 2 ? 1 : 0;
  const int tc = threadIdx.x & (kBlock / 2 - 1);
  const int TXh = TX / 2;
  const int cx = 2 * (tc % TXh), cy = tc / TXh;
  const bool own = tc < TXh * TY;
  T acc0[kColZ], acc1[kColZ];
#pragma unroll
  for (int z = 0; z < kColZ; ++z) acc0[z] = acc1[z] = (T)0;

  // weights: G2 lanes per particle, lane kr evaluates stencil row kr in x, y
  // and z with its coefficient row in registers
  constexpr int G2 = Lanes<P>::G2;
  const int kr = threadIdx.x % G2, pv = threadIdx.x / G2, per_pass = blockDim.x / G2;
  T crow[kMaxNu + 1];
  load_row(reinterpret_cast<const T*>(b.wtab), min(kr, P - 1), m, crow);
  for (int v0 = 0; v0 < total; v0 += kColBatch) {
    const int nb = min(kColBatch, total - v0);
    if (v0 > 0) __syncthreads();   // the previous batch has been consumed
    // the batch's particle records, at most one per thread, in one round of
    // loads (the weight loop below would otherwise wait for a load per pass)
    static_assert(kColBatch <= kBlock, "one record per thread");
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
      const int e = v0 + k;
      const int r = find_range(rpre, nr, e);
      const int i = rstart[r] + (e - rpre[r]);
      pq[k] = ld_quad<T>(b.s_fq, i);
      ppc[k] = gld(b.s_cell)[i];
      pcd[k] = rsh[r];
    }
    __syncthreads();
    for (int k = pv; k < nb; k += per_pass) {
      const Quad<T> f = pq[k];
      const int pc = ppc[k], code = pcd[k];
      // stencil origin c + shift - P/2 + 1 in tile coordinates, each in [-P+1, T)
      const int ox = (pc & 1023) + pc_sh[0][code >> 8] - P / 2 + 1 - x0;
      const int oy = ((pc >> 10) & 1023) + pc_sh[1][(code >> 4) & 15] - P / 2 + 1 - y0;
      const int oz = ((pc >> 20) & 1023) + pc_sh[2][code & 15] - P / 2 + 1 - z0;
      if (kr == 0) org[k] = (ox + 64) | ((oy + 64) << 8);
      T* w = wb + k * SW;
      // zeros first (z row, x padding), then the stencil rows over them (both
      // by this particle's lanes of one wavefront, so in this order)
      for (int z = kr; z < kColZ; z += G2) w[z] = (T)0;
      if (kr == 0) w[XO] = (T)0;
      if (kr == 1 % G2) w[XO + P + 1] = (T)0;
      if (kr < P) {
        w[XO + 1 + kr] = weight_reg<T, P>(g, crow, kr, f.fx);
        w[YO + kr] = weight_reg<T, P>(g, crow, kr, f.fy);
        const int zz = oz + kr;
        if ((unsigned)zz < (unsigned)kColZ) w[zz] = f.q * weight_reg<T, P>(g, crow, kr, f.fz);
      }
    }
    __syncthreads();
    // origins of 64 visits at a time, one per lane, broadcast by readlane;
    // all lanes stay active through the loop (readlane reads every lane's
    // value); each half of the workgroup takes every other visit
    for (int k0 = 0; k0 < nb; k0 += 64) {
      const int my_org = org[min(k0 + (int)(threadIdx.x & 63), nb - 1)];
      const int kn = min(64, nb - k0);
      for (int j = half; j < kn; j += 2) {
        const int o = __builtin_amdgcn_readlane(my_org, j);
        const int ox = (o & 255) - 64, oy = ((o >> 8) & 255) - 64;
        const int dx = cx - ox, dy = cy - oy;
        // columns cx, cx + 1 meet the stencil's x range [0, P) when dx in [-1, P)
        if (own && (unsigned)dy < (unsigned)P && (unsigned)(dx + 1) < (unsigned)(P + 1)) {
          const T* w = wb + (k0 + j) * SW;
          const T wy = w[YO + dy];
          const T a0 = w[XO + 1 + dx] * wy, a1 = w[XO + 2 + dx] * wy;
          const vec4<T>* wz4 = reinterpret_cast<const vec4<T>*>(w);
#pragma unroll
          for (int q = 0; q < kColZ / 4; ++q) {
            const vec4<T> v = wz4[q];
            acc0[4 * q] += a0 * v.x;
            acc0[4 * q + 1] += a0 * v.y;
            acc0[4 * q + 2] += a0 * v.z;
            acc0[4 * q + 3] += a0 * v.w;
            acc1[4 * q] += a1 * v.x;
            acc1[4 * q + 1] += a1 * v.y;
            acc1[4 * q + 2] += a1 * v.z;
            acc1[4 * q + 3] += a1 * v.w;
          }
        }
      }
    }
  }
  // the odd-visit half hands its sums to the even-visit half through LDS
  // (the weight records are consumed), which adds them in a fixed order
  __syncthreads();
  T* red = wb;   // kBlock / 2 threads x 2 kColZ values
  if (half) {
#pragma unroll
    for (int z = 0; z < kColZ; ++z) {
      red[z * (kBlock / 2) + tc] = acc0[z];
      red[(kColZ + z) * (kBlock / 2) + tc] = acc1[z];
    }
  }
  __syncthreads();
  if (!half && own && cy < ey) {
#pragma unroll
    for (int z = 0; z < kColZ; ++z) {
      acc0[z] += red[z * (kBlock / 2) + tc];
      acc1[z] += red[(kColZ + z) * (kBlock / 2) + tc];
    }
    T* grid = reinterpret_cast<T*>(b.grid);
    const long long base = ((long long)z0 * g.G[1] + y0 + cy) * g.G[0] + x0 + cx;
    const long long zs = (long long)g.G[0] * g.G[1];
#pragma unroll
    for (int z = 0; z < kColZ; ++z)
      if (z < ez) {
        if (cx < ex) gst(grid)[base + z * zs] = acc0[z];
        if (cx + 1 < ex) gst(grid)[base + z * zs + 1] = acc1[z];
      }
  }
  __syncthreads();
}

// The spread stage in the plan's mode: boxes to staging (folded afterwards)
// or clipped stencils straight into the grid.
template <typename T, int P>
__device__ __forceinline__ void stage_spread_mode(const GridGeom& g, const EvalBuffers& b, int item,
                                                  unsigned char* smem) {
  if (g.clip == 2) stage_spread_cols<T, P>(g, b, item, smem);
  else if (g.clip) stage_spread_clip<T, P>(g, b, item, smem);
  else stage_spread<T, P>(g, b, item, smem);
}

template <typename T, int P>
__global__ __launch_bounds__(kBlock) void spread_kernel(GridGeom g, EvalBuffers b) {
  extern __shared__ __align__(16) unsigned char smem[];
  stage_spread_mode<T, P>(g, b, work_item(g.xcd), smem);
}

// For one direction: the tile at offset d from tile t (wrapped in periodic
// directions), and the origin of its box in the unwrapped frame of tile t.
// Returns false if there is no such tile.
__device__ __forceinline__ bool box_of(const GridGeom& g, int dim, int t, int d, int* tile, int* org) {
  const int nt = g.nt[dim], G = g.G[dim];
  int u = t + d, shift = 0;
  while (u < 0) {
    if (!g.per[dim]) return false;
    u += nt;
    shift -= G;
  }
  while (u >= nt) {
    if (!g.per[dim]) return false;
    u -= nt;
    shift += G;
  }
  *tile = u;
  *org = u * g.T[dim] + shift - (g.P / 2 - 1);
  return true;
}

// Boxes (tile, origin) of one direction that intersect [x0, x0 + ext): the
// tiles at offsets d from tile t, periodic images included.  Offsets are
// scanned generously (a partial last tile in a periodic direction brings the
// images closer than T apart) and kept only if the box meets the tile.
__device__ __forceinline__ int fold_images(const GridGeom& g, int dim, int t, int x0, int ext, int* tl,
                                           int* org) {
  const int T = g.T[dim], RX = T + g.P - 1;
  int emin = T;
  if (g.per[dim]) emin = min(T, g.G[dim] - (g.nt[dim] - 1) * T);
  const int reach = 2 + (T + g.P) / max(emin, 1);
  int n = 0;
  for (int d = -reach; d <= reach; ++d) {
    int u, o;
    if (!box_of(g, dim, t, d, &u, &o)) continue;
    if (o < x0 + ext && o + RX > x0 && n < kMaxFoldImages) {
      tl[n] = u;
      org[n] = o;
      ++n;
    }
  }
  return n;
}

template <typename T>
__device__ __forceinline__ void stage_fold(const GridGeom& g, const EvalBuffers& b, int item) {
  const int t_id = item;
  const int tz = t_id / (g.nt[0] * g.nt[1]);
  const int ty = (t_id / g.nt[0]) % g.nt[1];
  const int tx = t_id % g.nt[0];
  const int x0 = tx * g.T[0], y0 = ty * g.T[1], z0 = tz * g.T[2];
  const int ex = min(g.T[0], g.G[0] - x0), ey = min(g.T[1], g.G[1] - y0), ez = min(g.T[2], g.G[2] - z0);
  const int RX = g.T[0] + g.P - 1, RY = g.T[1] + g.P - 1, RZ = g.T[2] + g.P - 1;
  const long long R3 = (long long)RX * RY * RZ;
  int tlx[kMaxFoldImages], olx[kMaxFoldImages], tly[kMaxFoldImages], oly[kMaxFoldImages], tlz[kMaxFoldImages], olz[kMaxFoldImages];
  const int nx = fold_images(g, 0, tx, x0, ex, tlx, olx);
  const int ny = fold_images(g, 1, ty, y0, ey, tly, oly);
  const int nz = fold_images(g, 2, tz, z0, ez, tlz, olz);
  const T* stg = reinterpret_cast<const T*>(b.stage);
  T* grid = reinterpret_cast<T*>(b.grid);
  // rows of the tile, 64 / TX rows per wavefront at a time
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, nwaves = blockDim.x / 64;
  const int rpw = 64 / g.T[0], sub = lane / g.T[0], lxo = lane - sub * g.T[0];
  const int nrows = ey * ez;
  if (sub >= rpw || lxo >= ex) return;
  for (int r0 = wave * rpw; r0 < nrows; r0 += nwaves * rpw) {
    const int row = r0 + sub;
    if (row >= nrows) break;
    const int x = x0 + lxo, y = y0 + row % ey, z = z0 + row / ey;
    T sum = 0;
    for (int kz = 0; kz < nz; ++kz) {
      const int bz = z - olz[kz];
      if (bz < 0 || bz >= RZ) continue;
      for (int ky = 0; ky < ny; ++ky) {
        const int by = y - oly[ky];
        if (by < 0 || by >= RY) continue;
        for (int kx = 0; kx < nx; ++kx) {
          const int bx = x - olx[kx];
          if (bx < 0 || bx >= RX) continue;
          const long long nt = ((long long)tlz[kz] * g.nt[1] + tly[ky]) * g.nt[0] + tlx[kx];
          sum += gld(stg)[nt * R3 + ((long long)bz * RY + by) * RX + bx];
        }
      }
    }
    gst(grid)[((long long)z * g.G[1] + y) * g.G[0] + x] = sum;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fold_kernel(GridGeom g, EvalBuffers b) {
  stage_fold<T>(g, b, work_item(g.xcd));
}

template <typename T>
size_t spread_lds(const GridGeom& g) {
  const int P = g.P, nw = kBlock / 64;
  if (g.clip == 2) {
    const size_t sw = (size_t)(kColZ + 2 * P + 2 + 3) / 4 * 4;   // ColLayout::SW
    return sizeof(int) * (3 * kMaxClipRanges + 4 + kColBatch) +
           sizeof(T) * (kColBatch * sw > (size_t)kBlock * kColZ ? kColBatch * sw : (size_t)kBlock * kColZ) +
           kColBatch * (4 * sizeof(T) + 2 * sizeof(int)) + 64;
  }
  if (g.clip) {
    const size_t T3 = (size_t)g.T[0] * g.T[1] * g.T[2];
    return 8 * T3 + sizeof(T) * ((size_t)nw * g.chunk * (3 * P + 4)) +
           sizeof(int) * (3 * kMaxClipRanges + 4 + nw * g.chunk * 3 + 4) + 64;
  }
  const size_t R3 = (size_t)(g.T[0] + P - 1) * (g.T[1] + P - 1) * (g.T[2] + P - 1);
  return 8 * R3 + sizeof(T) * ((size_t)nw * g.chunk * (3 * P + 4)) +
         sizeof(int) * (2 * kMaxOwnRanges + 4 + nw * g.chunk * 3 + 4) + 64;
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

hipError_t launch_fold(const GridGeom& g, const EvalBuffers& b, bool f64, hipStream_t st) {
  const int ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  if (f64)
    fold_kernel<double><<<dim3(ntiles), dim3(kBlock), 0, st>>>(g, b);
  else
    fold_kernel<float><<<dim3(ntiles), dim3(kBlock), 0, st>>>(g, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gathering, trapezoidal rule of Eq. (complete_integral), and the gradient of
// Eq. (force-method-1).  One workgroup per tile stages the tile's stencil
// region of the grid in LDS and takes the particles anchored in the tile.
// A group of P lanes serves one particle; lane iz owns the z-plane iz of the
// stencil, evaluates row iz of the three weight vectors, contracts its plane
// separably (x, then y) and the group sums the planes with shuffles.
// ---------------------------------------------------------------------------
template <typename T, int P, int MODE = GM_ALL>
__device__ __forceinline__ void stage_gather(const GridGeom& g, const EvalBuffers& b, T* __restrict__ phi,
                             T* __restrict__ force, int out_grad, double self_coef, int item,
                             unsigned char* smem, int comp = 0) {
  constexpr bool GRAD = MODE == GM_ALL;
  constexpr int G2 = GatherLanes<P, T>::G, PPW = GatherLanes<P, T>::PPW;
  const int TX = g.T[0], TY = g.T[1], TZ = g.T[2];
  const int t_id = item;
  const int tz = t_id / (g.nt[0] * g.nt[1]);
  const int ty = (t_id / g.nt[0]) % g.nt[1];
  const int tx = t_id % g.nt[0];
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int ex = min(TX, g.G[0] - x0), ey = min(TY, g.G[1] - y0), ez = min(TZ, g.G[2] - z0);
  const int RX = TX + P - 1, RY = TY + P - 1, RZ = TZ + P - 1;
  const int m = g.nu + 1;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nwaves = blockDim.x / 64;

  T* reg = reinterpret_cast<T*>(smem);                       // RX*RY*RZ
  int* rstart = reinterpret_cast<int*>(reg + RX * RY * RZ);   // kMaxOwnRanges
  int* rpre = rstart + kMaxOwnRanges;                         // kMaxOwnRanges + 1
  T* wsh = reinterpret_cast<T*>(rpre + kMaxOwnRanges + 4);    // nwaves * PPW * 4P
  Quad<T>* rq = reinterpret_cast<Quad<T>*>(wsh + nwaves * PPW * 4 * P);   // kGatherBatch records
  int* rc = reinterpret_cast<int*>(rq + kGatherBatch);        // kGatherBatch cells
  int* ri = rc + kGatherBatch;                                // kGatherBatch input indices
  __shared__ double ewave[kGatherBlock / 64];

  // particles anchored in this tile: sub-bins of the tile
  int sx[2] = {x0 / kSB, (x0 + ex - 1) / kSB}, sy[2] = {y0 / kSB, (y0 + ey - 1) / kSB},
      sz[2] = {z0 / kSB, (z0 + ez - 1) / kSB};
  const int nr = (sz[1] - sz[0] + 1) * (sy[1] - sy[0] + 1);
  const int total = build_ranges(g, b, sz, 1, sy, 1, sx, 1, rstart, rpre);
  if (total == 0) {
    if (MODE != GM_COMP && threadIdx.x == 0) gst(b.epart)[t_id] = 0.0;
    return;
  }

  // particle records of a batch, one per thread in one round of loads
  auto load_batch = [&](int b0) {
    const int nb = min(kGatherBatch, total - b0);
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
      const int e = b0 + k;
      const int r = find_range(rpre, nr, e);
      const int i = rstart[r] + (e - rpre[r]);
      rq[k] = ld_quad<T>(b.s_fq, i);
      rc[k] = gld(b.s_cell)[i];
      ri[k] = gld(b.s_idx)[i];
    }
  };
  load_batch(0);   // in flight together with the region below

  // stage the stencil region [x0 - P/2 + 1, x0 + TX + P/2 - 1] of the grid:
  // rows of RX points are read as 16-byte chunks of V points (one chunk per
  // lane, LR lanes per row, 64 / LR rows per wavefront at a time); a chunk
  // inside [0, G0) is one load, a chunk across a periodic or free x boundary
  // is read point by point.  The LDS rows keep pitch RX (a padded pitch would
  // put the z planes of one particle's lanes on the same banks in the
  // contraction below), so chunks are written point by point.  Rows advance
  // by additions: the row index, its (y, z) place in the region and the
  // wrapped grid coordinates need no division per load.
  const T* grid = reinterpret_cast<const T*>(b.grid);
  const int rx = x0 - P / 2 + 1, ry = y0 - P / 2 + 1, rz = z0 - P / 2 + 1;
  {
    constexpr int V = 16 / (int)sizeof(T);
    constexpr int U = 8;  // rows in flight per lane
    const int LR = (RX + V - 1) / V;
    const int rpw = 64 / LR, sub = lane / LR, cpos = lane - sub * LR;
    const int nrows = RY * RZ, step = nwaves * rpw;
    const int G0 = g.G[0], G1 = g.G[1], G2y = g.G[2];
    if (sub < rpw) {
      const int xs = rx + cpos * V;                    // unwrapped x of the chunk's first point
      const bool whole = xs >= 0 && xs + V <= G0;      // no x boundary inside the chunk
      int gxv[V];
      bool okxv[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        okxv[e] = cpos * V + e < RX;
        gxv[e] = wrap_coord(g, 0, xs + e, &okxv[e]);
      }
      const int step_q = step / RY, step_r = step - step_q * RY;
      int row = wave * rpw + sub;
      int py = row % RY, pz = row / RY;
      auto wrapped = [&](int d, int c, int G, bool* ok) {
        if (g.per[d]) {
          while (c >= G) c -= G;
          while (c < 0) c += G;
        } else {
          *ok = *ok && c >= 0 && c < G;
        }
        return c;
      };
      using C16 = T __attribute__((ext_vector_type(V)));   // one 16-byte chunk
      while (row < nrows) {
        C16 v[U];
        int lrow[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          v[u] = (C16)(T)0;
          lrow[u] = row < nrows ? row : -1;
          if (row < nrows) {
            bool ok = true;
            const int gy = wrapped(1, ry + py, G1, &ok), gz = wrapped(2, rz + pz, G2y, &ok);
            if (ok) {
              const T* src = grid + ((long long)gz * G1 + gy) * G0;
              if (whole) {
                // point-aligned, not chunk-aligned in memory: copied, not dereferenced as C16
                __builtin_memcpy(&v[u], src + xs, sizeof(C16));
              } else {
#pragma unroll
                for (int e = 0; e < V; ++e)
                  if (okxv[e]) v[u][e] = gld(src)[gxv[e]];
              }
            }
          }
          row += step;
          py += step_r;
          pz += step_q;
          if (py >= RY) {
            py -= RY;
            ++pz;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (lrow[u] >= 0) {
            T* dst = reg + lrow[u] * RX + cpos * V;
#pragma unroll
            for (int e = 0; e < V; ++e)
              if (cpos * V + e < RX) dst[e] = v[u][e];
          }
      }
    }
  }

  const int p = lane / G2, iz = lane % G2;
  // coefficient rows (values, derivatives) of stencil row iz in registers
  T crow[kMaxNu + 1], drow[kMaxNu + 1];
  {
    const T* wt = reinterpret_cast<const T*>(b.wtab);
    load_row(wt, min(iz, P - 1), m, crow);
    load_row(wt + P * m, min(iz, P - 1), m, drow);
  }
  __syncthreads();

  T* wp = wsh + (wave * PPW + p) * 4 * P;    // wx | dwx | wy | dwy of this lane's particle
  const T sc = (T)g.scale;
  double eacc = 0.0;
  for (int b0 = 0; b0 < total; b0 += kGatherBatch) {
    if (b0 > 0) {
      __syncthreads();
      load_batch(b0);
      __syncthreads();
    }
    const int nb = min(kGatherBatch, total - b0);
    for (int base = wave * PPW; base < nb; base += nwaves * PPW) {
      const int k = base + p;
      const bool valid = p < PPW && k < nb;   // lanes past PPW G2 serve no particle
      const Quad<T> f = valid ? rq[k] : Quad<T>{0, 0, 0, 0};
      const int pc = valid ? rc[k] : 0;
      const int lx = (pc & 1023) - x0, ly = ((pc >> 10) & 1023) - y0, lz = ((pc >> 20) & 1023) - z0;
      T wz = 0, dwz = 0;
      if (valid && iz < P) {
        wp[iz] = weight_reg<T, P>(g, crow, iz, f.fx);
        wp[2 * P + iz] = weight_reg<T, P>(g, crow, iz, f.fy);
        wz = weight_reg<T, P>(g, crow, iz, f.fz);
        if constexpr (GRAD) {
          wp[P + iz] = dweight_reg<T, P>(g, drow, iz, f.fx);
          wp[3 * P + iz] = dweight_reg<T, P>(g, drow, iz, f.fy);
          dwz = dweight_reg<T, P>(g, drow, iz, f.fz);
        }
      }
      wave_sync();
      T ph = 0, gx = 0, gy = 0, gz = 0;
      if (valid && iz < P) {
        T wx[P], dwx[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
          wx[q] = wp[q];
          dwx[q] = GRAD ? wp[P + q] : (T)0;
        }
        T s00 = 0, s01 = 0, s10 = 0;
        const T* plane = reg + (long long)(lz + iz) * RX * RY + (long long)ly * RX + lx;
#pragma unroll
        for (int iy = 0; iy < P; ++iy) {
          const T* row = plane + iy * RX;
          T r0 = 0, r1 = 0;
#pragma unroll
          for (int ix = 0; ix < P; ++ix) {
            const T v = row[ix];
            r0 += wx[ix] * v;
            if constexpr (GRAD) r1 += dwx[ix] * v;
          }
          const T wy = wp[2 * P + iy];
          s00 += wy * r0;
          if constexpr (GRAD) {
            const T dwy = wp[3 * P + iy];
            s01 += dwy * r0;
            s10 += wy * r1;
          }
        }
        ph = wz * s00;
        gx = wz * s10;
        gy = wz * s01;
        gz = dwz * s00;
      }
      ph = segment_sum<G2>(ph, iz);
      if constexpr (GRAD) {
        gx = segment_sum<G2>(gx, iz);
        gy = segment_sum<G2>(gy, iz);
        gz = segment_sum<G2>(gz, iz);
      }
      if (valid && iz == 0) {
        const int idx = ri[k];
        if constexpr (MODE == GM_COMP) {
          // force method 2: the grid holds the derivative along comp
          const T f0 = out_grad ? (T)1 : -f.q;
          gst(force)[3 * idx + comp] = f0 * sc * ph;
        } else {
          const T pv = sc * ph + (T)(self_coef * (double)f.q);
          if (phi) gst(phi)[idx] = pv;
          if (GRAD && force) {
            const T f0 = out_grad ? (T)1 : -f.q;
            const auto fo = gst(force);
            fo[3 * idx] = f0 * sc * gx;
            fo[3 * idx + 1] = f0 * sc * gy;
            fo[3 * idx + 2] = f0 * sc * gz;
          }
          eacc += (double)f.q * (double)pv;
        }
      }
      wave_sync();
    }
  }
  if constexpr (MODE != GM_COMP) {
    eacc = warp_sum(eacc);
    if (lane == 0) ewave[wave] = eacc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < nwaves; ++w) s += ewave[w];
      gst(b.epart)[t_id] = s;
    }
  }
  __syncthreads();
}

template <typename T, int P, int MODE>
__global__ __launch_bounds__(kGatherBlock) void gather_kernel(GridGeom g, EvalBuffers b, T* __restrict__ phi,
                                                        T* __restrict__ force, int out_grad,
                                                        double self_coef, int comp) {
  extern __shared__ __align__(16) unsigned char smem[];
  stage_gather<T, P, MODE>(g, b, phi, force, out_grad, self_coef, work_item(g.xcd), smem, comp);
}

template <typename T>
size_t gather_lds(const GridGeom& g) {
  const int P = g.P, m = g.nu + 1, nw = kGatherBlock / 64;
  const int G = P < 2 ? 2 : P;   // GatherLanes<P, T>
  const int ppw = sizeof(T) == 8 && 64 / G > 4 ? 4 : 64 / G;
  const size_t R = (size_t)(g.T[0] + P - 1) * (g.T[1] + P - 1) * (g.T[2] + P - 1);
  (void)m;
  return sizeof(T) * (R + (size_t)nw * ppw * 4 * P + 4 * kGatherBatch) +
         sizeof(int) * (2 * kMaxOwnRanges + 4 + 2 * kGatherBatch) + 64;
}

template <typename T, int P>
static void gather_launch(const GridGeom& g, const EvalBuffers& b, T* phi, T* force, int out_grad,
                          double self_coef, hipStream_t st, int mode, int comp) {
  const int ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  const dim3 grid(ntiles), block(kGatherBlock);
  const size_t lds = gather_lds<T>(g);
  switch (mode) {
    case GM_PHI:
      gather_kernel<T, P, GM_PHI><<<grid, block, lds, st>>>(g, b, phi, force, out_grad, self_coef, comp);
      break;
    case GM_COMP:
      gather_kernel<T, P, GM_COMP><<<grid, block, lds, st>>>(g, b, phi, force, out_grad, self_coef, comp);
      break;
    default:
      gather_kernel<T, P, GM_ALL><<<grid, block, lds, st>>>(g, b, phi, force, out_grad, self_coef, comp);
      break;
  }
}

template <typename T>
static hipError_t gather_dispatch(const GridGeom& g, const EvalBuffers& b, void* phi, void* force,
                                  int out_grad, double self_coef, hipStream_t st, int mode, int comp) {
  T* p = reinterpret_cast<T*>(phi);
  T* f = reinterpret_cast<T*>(force);
  switch (g.P) {
    case 2: gather_launch<T, 2>(g, b, p, f, out_grad, self_coef, st, mode, comp); break;
    case 4: gather_launch<T, 4>(g, b, p, f, out_grad, self_coef, st, mode, comp); break;
    case 6: gather_launch<T, 6>(g, b, p, f, out_grad, self_coef, st, mode, comp); break;
    case 8: gather_launch<T, 8>(g, b, p, f, out_grad, self_coef, st, mode, comp); break;
    case 10: gather_launch<T, 10>(g, b, p, f, out_grad, self_coef, st, mode, comp); break;
    case 12: gather_launch<T, 12>(g, b, p, f, out_grad, self_coef, st, mode, comp); break;
    case 14: gather_launch<T, 14>(g, b, p, f, out_grad, self_coef, st, mode, comp); break;
    case 16: gather_launch<T, 16>(g, b, p, f, out_grad, self_coef, st, mode, comp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t gather_lds_bytes(const GridGeom& g, bool f64) {
  return f64 ? gather_lds<double>(g) : gather_lds<float>(g);
}

hipError_t launch_gather(const GridGeom& g, const EvalBuffers& b, bool f64, void* phi, void* force,
                         int out_grad, double self_coef, hipStream_t st, int mode, int comp) {
  return f64 ? gather_dispatch<double>(g, b, phi, force, out_grad, self_coef, st, mode, comp)
             : gather_dispatch<float>(g, b, phi, force, out_grad, self_coef, st, mode, comp);
}

// E = 1/2 sum of the per-tile partials of q phi, in a fixed order (FP64).
__device__ __forceinline__ void stage_energy(const double* __restrict__ epart, int n, double* __restrict__ energy) {
  __shared__ double es[kBlock];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a += epart[i];
  es[threadIdx.x] = a;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) es[threadIdx.x] += es[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && energy) *energy = 0.5 * es[0];
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void energy_kernel(const double* __restrict__ epart, int n,
                                                        double* __restrict__ energy) {
  stage_energy(epart, n, energy);
}

hipError_t launch_energy(const GridGeom& g, const EvalBuffers& b, double* energy, double self_e,
                         hipStream_t st) {
  (void)self_e;
  const int ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  energy_kernel<<<dim3(1), dim3(kBlock), 0, st>>>(b.epart, ntiles, energy);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void zero_kernel(GridGeom g, EvalBuffers b);

hipError_t launch_zero(const GridGeom& g, const EvalBuffers& b, hipStream_t st) {
  zero_kernel<<<dim3(scan_blocks(g)), dim3(kBlock), 0, st>>>(g, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint combinations (the chain rule of the autograd layer), FP64 arithmetic.
// E = 1/2 sum q phi with phi = A q symmetric in q gives dE/dq = phi and
// dE/dx_m = q_m grad phi(x_m) (Section 7.2); for a potential cotangent g,
// dL/dq = A g and dL/dx_m = g_m grad phi(x_m) + q_m grad (A g)(x_m).
// ---------------------------------------------------------------------------
template <typename Tin, typename T>
__global__ __launch_bounds__(kBlock) void energy_vjp_kernel(long N, const double* __restrict__ gE,
                                                            const Tin* __restrict__ q, const T* __restrict__ phi,
                                                            const T* __restrict__ grad, Tin* __restrict__ gx,
                                                            Tin* __restrict__ gq) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const double s = *gE;
  if (gx) {
    const double sq = s * (double)q[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) gx[3 * i + k] = (Tin)(sq * (double)grad[3 * i + k]);
  }
  if (gq) gq[i] = (Tin)(s * (double)phi[i]);
}

template <typename Tin, typename T>
__global__ __launch_bounds__(kBlock) void potential_vjp_kernel(long N, const Tin* __restrict__ q,
                                                               const Tin* __restrict__ g, const T* __restrict__ grad,
                                                               const T* __restrict__ ag, const T* __restrict__ agrad,
                                                               Tin* __restrict__ gx, Tin* __restrict__ gq) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  if (gx) {
    const double gi = (double)g[i], qi = (double)q[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) gx[3 * i + k] = (Tin)(gi * (double)grad[3 * i + k] + qi * (double)agrad[3 * i + k]);
  }
  if (gq) gq[i] = (Tin)ag[i];
}

template <typename Tin, typename T>
static void energy_vjp_t(long N, const double* gE, const void* q, const void* phi, const void* grad, void* gx,
                         void* gq, hipStream_t st) {
  energy_vjp_kernel<Tin, T><<<dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, st>>>(
      N, gE, (const Tin*)q, (const T*)phi, (const T*)grad, (Tin*)gx, (Tin*)gq);
}

template <typename Tin, typename T>
static void potential_vjp_t(long N, const void* q, const void* g, const void* grad, const void* ag, const void* agrad,
                            void* gx, void* gq, hipStream_t st) {
  potential_vjp_kernel<Tin, T><<<dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, st>>>(
      N, (const Tin*)q, (const Tin*)g, (const T*)grad, (const T*)ag, (const T*)agrad, (Tin*)gx, (Tin*)gq);
}

hipError_t launch_energy_vjp(long N, bool in_f32, bool f64, const double* gE, const void* q, const void* phi,
                             const void* grad, void* gx, void* gq, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (in_f32) f64 ? energy_vjp_t<float, double>(N, gE, q, phi, grad, gx, gq, st)
                  : energy_vjp_t<float, float>(N, gE, q, phi, grad, gx, gq, st);
  else f64 ? energy_vjp_t<double, double>(N, gE, q, phi, grad, gx, gq, st)
           : energy_vjp_t<double, float>(N, gE, q, phi, grad, gx, gq, st);
  return hipGetLastError();
}

hipError_t launch_potential_vjp(long N, bool in_f32, bool f64, const void* q, const void* g, const void* grad,
                                const void* ag, const void* agrad, void* gx, void* gq, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (in_f32) f64 ? potential_vjp_t<float, double>(N, q, g, grad, ag, agrad, gx, gq, st)
                  : potential_vjp_t<float, float>(N, q, g, grad, ag, agrad, gx, gq, st);
  else f64 ? potential_vjp_t<double, double>(N, q, g, grad, ag, agrad, gx, gq, st)
           : potential_vjp_t<double, float>(N, q, g, grad, ag, agrad, gx, gq, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched evaluation: many systems of uneven size and periodicity.  Each stage
// of the path is one launch over the work items of all systems (a work item is
// one block-sized piece of one system: a particle block, a scan block, a tile
// or a pencil group); consecutive launches on the stream order the stages.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stage_zero(const GridGeom& g, const EvalBuffers& b, int item) {
  const int n = g.nsb[0] * g.nsb[1] * g.nsb[2];
  for (int k = threadIdx.x; k < kScanBlock; k += blockDim.x) {
    const int i = item * kScanBlock + k;
    if (i < n) b.sb_count[i] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void zero_kernel(GridGeom g, EvalBuffers b) { stage_zero(g, b, blockIdx.x); }

template <typename T, int P>
__device__ __forceinline__ void run_batch_stage(int st, const SysDesc& S, int sys_id, int li, const BatchIO& io,
                                unsigned char* smem) {
  switch (st) {
    case BS_ZERO:
      stage_zero(S.g, S.b, li);
      break;
    case BS_BIN:
      if (io.in_f32)
        stage_bin<float, T>(S.g, S.b, S.N, reinterpret_cast<const float*>(io.xyz) + 3 * S.off,
                            reinterpret_cast<const float*>(io.q) + S.off, li);
      else
        stage_bin<double, T>(S.g, S.b, S.N, reinterpret_cast<const double*>(io.xyz) + 3 * S.off,
                             reinterpret_cast<const double*>(io.q) + S.off, li);
      break;
    case BS_SCAN1:
      stage_scan1(S.g, S.b, li);
      break;
    case BS_SCAN2:
      stage_scan2(S.g, S.b, S.nblk_bin, S.check_neutral && !io.allow_nonneutral, li, S.nscan);
      break;
    case BS_SCATTER:
      stage_scatter<T>(S.b, S.N, li);
      break;
    case BS_ORDER:
      stage_order<T>(S.b, S.g.nsb[0] * S.g.nsb[1] * S.g.nsb[2], li);
      break;
    case BS_SPREAD:
      stage_spread_mode<T, P>(S.g, S.b, li, smem);
      break;
    case BS_FOLD:
      stage_fold<T>(S.g, S.b, li);
      break;
    case BS_GATHER: {
      T* phi = io.phi ? reinterpret_cast<T*>(io.phi) + S.off : nullptr;
      T* force = io.force ? reinterpret_cast<T*>(io.force) + 3 * S.off : nullptr;
      stage_gather<T, P>(S.g, S.b, phi, force, io.out_grad, io.add_self ? S.self_coef : 0.0, li, smem);
      break;
    }
    case BS_ENERGY:
      stage_energy(S.b.epart, S.ntiles, io.energy ? io.energy + sys_id : nullptr);
      break;
    default:
      break;
  }
}

// One stage of the batch for all systems: block b is work item b of the stage,
// counted over the systems in order.  No block waits on another.  The stage
// is a template argument so that each stage's kernel carries only its own
// registers and LDS.
template <typename T, int P, int ST>
__global__ __launch_bounds__(stage_block(ST)) void batch_stage_kernel(const SysDesc* __restrict__ sys, int nsys,
                                                             const int* __restrict__ off, BatchIO io, int xcd) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int* o = off + ST * (nsys + 1);
  const int item = work_item(xcd);
  // the system owning this item: last s with o[s] <= item
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (o[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);  // uniform: keeps the descriptor in scalar registers
  run_batch_stage<T, P>(ST, sys[lo], lo, item - o[lo], io, smem);
}

template <typename T, int P, int ST>
static void batch_launch_one(const SysDesc* sys, int nsys, const int* off, const int* items, const BatchIO& io,
                             const size_t* lds, hipStream_t st, hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[ST], st);
  if constexpr (ST >= BS_FFT0 && ST <= BS_FFT4) {
    const int pass = ST - BS_FFT0;
    const bool wide = (io.fft_wide >> pass) & 1;
    // records of earlier transform lists come first
    long first = 0;
    for (int l = BS_COUNT; l < fft_list(ST, 0); ++l) first += items[l];
    for (int k = 0; k < kFftKinds; ++k) {
      if (items[fft_list(ST, k)] > 0)
        launch_batch_fft(sizeof(T) == 8, k, wide, sys, io.fft_rec + first, pass, items[fft_list(ST, k)], lds[ST],
                         io.xcd_fft, st);
      first += items[fft_list(ST, k)];
    }
  } else {
    if (items[ST] > 0)
      batch_stage_kernel<T, P, ST><<<dim3(items[ST]), dim3(stage_block(ST)), lds[ST], st>>>(
          sys, nsys, off, io, (ST == BS_SPREAD || ST == BS_FOLD || ST == BS_GATHER) ? io.xcd_tiles : 0);
  }
}

template <typename T, int P>
static void batch_launch_t(const SysDesc* sys, int nsys, const int* off, const int* items, const BatchIO& io,
                           const size_t* lds, hipStream_t st, hipEvent_t* ev) {
  batch_launch_one<T, P, BS_ZERO>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_BIN>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_SCAN1>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_SCAN2>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_SCATTER>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_ORDER>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_SPREAD>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_FOLD>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_FFT0>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_FFT0 + 1>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_FFT0 + 2>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_FFT0 + 3>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_FFT0 + 4>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_GATHER>(sys, nsys, off, items, io, lds, st, ev);
  batch_launch_one<T, P, BS_ENERGY>(sys, nsys, off, items, io, lds, st, ev);
  if (ev) (void)hipEventRecord(ev[BS_COUNT], st);
}

hipError_t launch_batch(int P, bool f64, const SysDesc* sys, int nsys, const int* off, const int* items,
                        const BatchIO& io, const size_t* lds, hipStream_t st, hipEvent_t* ev) {
  switch (P) {
    case 4: f64 ? batch_launch_t<double, 4>(sys, nsys, off, items, io, lds, st, ev)
                : batch_launch_t<float, 4>(sys, nsys, off, items, io, lds, st, ev); break;
    case 6: f64 ? batch_launch_t<double, 6>(sys, nsys, off, items, io, lds, st, ev)
                : batch_launch_t<float, 6>(sys, nsys, off, items, io, lds, st, ev); break;
    case 8: f64 ? batch_launch_t<double, 8>(sys, nsys, off, items, io, lds, st, ev)
                : batch_launch_t<float, 8>(sys, nsys, off, items, io, lds, st, ev); break;
    case 10: f64 ? batch_launch_t<double, 10>(sys, nsys, off, items, io, lds, st, ev)
                 : batch_launch_t<float, 10>(sys, nsys, off, items, io, lds, st, ev); break;
    case 12: f64 ? batch_launch_t<double, 12>(sys, nsys, off, items, io, lds, st, ev)
                 : batch_launch_t<float, 12>(sys, nsys, off, items, io, lds, st, ev); break;
    default: return hipErrorInvalidValue;
  }
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

// Octant (Mt+1)^3 of the real, even effective Green's function, index
// [kz][ky][kx] (kx fastest, as the grid).
template <typename T>
__global__ void g0p_fold_kernel(const cx<double>* full, int Mt, T* table) {
  const int n = 2 * Mt, m = Mt + 1;
  const long long N = (long long)m * m * m;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)((e / m) % m), k = (int)(e / ((long long)m * m));
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
