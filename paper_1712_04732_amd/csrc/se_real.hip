// Real-space part of the Ewald sum on the GPU, Eq. (real_space_ewald):
//
//   phi^R_m = sum over lattice images p of P_D and charges n, skipping n = m
//             at p = 0, of q_n erfc(xi r) / r,   r = |x_m - x_n + p| < rc,
//
// with its gradient d phi^R / d x_m (Section 7.2 differentiates every part of
// the split in the same way).  It completes the k-space result of se_eval
// into the full potential of Eq. (potential_split).
//
// Cell list: the box (a cube, or a rectangular box with a side per
// direction) is cut into c_d cells of side h_d = L_d/c_d >= rc/s_d
// per direction; every charge within rc of a target lies in the
// (2s_x+1)(2s_y+1)(2s_z+1) cells around the target's cell (periodic
// directions wrap with an image shift, free directions stop at the box).  Cells whose nearest points are rc or more
// apart are skipped.  One wavefront serves one cell: its lanes hold the
// cell's targets (several lanes per target when the cell is small); each
// neighbour chunk of 64 charges is loaded one per lane, the charges within rc
// of the target cell's box are packed into LDS, and every lane reads them
// back from there in the pair loop.  Charges are ordered by cell, and inside a cell by
// input index, so the sums are reproducible run to run.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/se.h"
#include "se_device.h"

namespace se {
namespace {

constexpr int kRsBlock = 256;       // threads of the bin, scan, order and energy kernels
constexpr int kRsScanItems = 1024;  // cells per block of the cell-count scan
constexpr int kRsSortMax = 2048;    // most charges of a cell sorted by input index
constexpr int kRsMaxCells = 160;    // most cells per direction

struct RsGeom {
  int D;           // periodic directions: x; x, y; x, y, z
  int c[3], s[3];  // cells and neighbour span in cells, per direction
  double L[3];     // box side per direction
  double h[3];     // cell side per direction, L[d] / c[d]
  double rc, xi;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// LDS writes of a wavefront made visible to its other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wrap a periodic coordinate into [0, L).
__device__ __forceinline__ double wrap_periodic(double x, double L, double invL) {
  double w = x - L * floor(x * invL);
  if (w >= L) w -= L;
  if (w < 0.0) w = 0.0;
  return w;
}

__device__ __forceinline__ int cell_coord(double w, double inv_h, int c) {
  const int i = (int)(w * inv_h);
  return i < 0 ? 0 : (i >= c ? c - 1 : i);
}

// Position of charge i, wrapped in the periodic directions; bit 1 of *bad for
// a non-finite value, bit 2 for a free coordinate outside [0, L).
template <typename Tin>
__device__ __forceinline__ void load_wrapped(const Tin* xyz, const Tin* q, long i, const RsGeom& g, double w[3],
                                             double* qi, int* bad) {
  *qi = (double)gld(q)[i];
  if (!isfinite(*qi)) *bad |= 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x = (double)gld(xyz)[3 * i + d];
    if (!isfinite(x)) {
      *bad |= 1;
      w[d] = 0.0;
    } else if (d < g.D) {
      w[d] = wrap_periodic(x, g.L[d], 1.0 / g.L[d]);
    } else {
      if (!(x >= 0.0 && x < g.L[d])) *bad |= 2;
      w[d] = x < 0.0 ? 0.0 : (x >= g.L[d] ? 0.0 : x);
    }
  }
}

// Cell of every charge and its arrival slot in that cell.
template <typename Tin>
__global__ __launch_bounds__(kRsBlock) void rs_bin_kernel(RsGeom g, long N, const Tin* __restrict__ xyz,
                                                          const Tin* __restrict__ q, int* __restrict__ cnt,
                                                          int* __restrict__ cell_of, int* __restrict__ slot,
                                                          int* __restrict__ status) {
  const long i = (long)blockIdx.x * kRsBlock + threadIdx.x;
  if (i >= N) return;
  double w[3], qi;
  int bad = 0;
  load_wrapped(xyz, q, i, g, w, &qi, &bad);
  if (bad) atomicOr(status, bad);
  const int cell = (cell_coord(w[2], g.c[2] / g.L[2], g.c[2]) * g.c[1] + cell_coord(w[1], g.c[1] / g.L[1], g.c[1])) *
                       g.c[0] +
                   cell_coord(w[0], g.c[0] / g.L[0], g.c[0]);
  gst(cell_of)[i] = cell;
  gst(slot)[i] = atomicAdd(cnt + cell, 1);
}

// Exclusive scan of the cell counts in three launches: block sums, a scan of
// the block sums in one workgroup, then each block's scan plus its offset.
__device__ __forceinline__ int block_scan_excl(int v, int* sh, int* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kRsBlock; o <<= 1) {
    const int a = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const int incl = sh[t];
  *total = sh[kRsBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kRsBlock) void rs_scan_sums_kernel(const int* __restrict__ cnt, int ncell,
                                                                int* __restrict__ bsum) {
  __shared__ int sh[kRsBlock];
  constexpr int per = kRsScanItems / kRsBlock;
  const int base = blockIdx.x * kRsScanItems + threadIdx.x * per;
  int v = 0;
#pragma unroll
  for (int k = 0; k < per; ++k)
    if (base + k < ncell) v += gld(cnt)[base + k];
  int total;
  (void)block_scan_excl(v, sh, &total);
  if (threadIdx.x == 0) gst(bsum)[blockIdx.x] = total;
}

__global__ __launch_bounds__(kRsBlock) void rs_scan_top_kernel(int* __restrict__ bsum, int nb) {
  __shared__ int sh[kRsBlock];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kRsBlock) {
    const int b = b0 + (int)threadIdx.x;
    const int v = b < nb ? bsum[b] : 0;
    int total;
    const int ex = block_scan_excl(v, sh, &total);
    if (b < nb) bsum[b] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kRsBlock) void rs_scan_apply_kernel(const int* __restrict__ cnt, int ncell,
                                                                 const int* __restrict__ bsum,
                                                                 int* __restrict__ start, long N) {
  __shared__ int sh[kRsBlock];
  constexpr int per = kRsScanItems / kRsBlock;
  const int base = blockIdx.x * kRsScanItems + threadIdx.x * per;
  int v[per], sum = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    v[k] = base + k < ncell ? gld(cnt)[base + k] : 0;
    sum += v[k];
  }
  int total;
  int run = block_scan_excl(sum, sh, &total) + gld(bsum)[blockIdx.x];
#pragma unroll
  for (int k = 0; k < per; ++k) {
    if (base + k < ncell) gst(start)[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) gst(start)[ncell] = (int)N;
}

__global__ __launch_bounds__(kRsBlock) void rs_scatter_kernel(long N, const int* __restrict__ cell_of,
                                                              const int* __restrict__ slot,
                                                              const int* __restrict__ start,
                                                              int* __restrict__ sidx) {
  const long i = (long)blockIdx.x * kRsBlock + threadIdx.x;
  if (i >= N) return;
  gst(sidx)[gld(start)[gld(cell_of)[i]] + gld(slot)[i]] = (int)i;
}

// One workgroup per cell: sort the cell's input indices (bitonic, in LDS;
// cells of more than kRsSortMax charges keep their arrival order), then
// store the cell's charges in that order as records {x, y, z, q} with the
// position taken from the cell's corner (so differences of nearby charges
// keep the precision of the cell side, not of the box), and the charge's x
// cell index in scx.  FP32 records come with an FP64 copy of the same
// cell-relative position in spos64 (null for FP64 records).
template <typename T, typename Tin>
__global__ __launch_bounds__(kRsBlock) void rs_order_kernel(RsGeom g, const Tin* __restrict__ xyz,
                                                            const Tin* __restrict__ q,
                                                            const int* __restrict__ start, int* __restrict__ sidx,
                                                            vec4<T>* __restrict__ spos, int* __restrict__ scx,
                                                            vec4<double>* __restrict__ spos64) {
  __shared__ int key[kRsSortMax];
  const int cell = blockIdx.x;
  const int j0 = start[cell], j1 = start[cell + 1], n = j1 - j0;
  if (n <= 0) return;
  const int cx = cell % g.c[0], cy = (cell / g.c[0]) % g.c[1], cz = cell / (g.c[0] * g.c[1]);
  if (n > 1 && n <= kRsSortMax) {
    int m = 1;
    while (m < n) m <<= 1;
    for (int i = threadIdx.x; i < m; i += kRsBlock) key[i] = i < n ? sidx[j0 + i] : 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < m; i += kRsBlock) {
          const int p = i ^ j;
          if (p > i) {
            const int a = key[i], b = key[p];
            const bool up = (i & k) == 0;
            if (up ? a > b : a < b) {
              key[i] = b;
              key[p] = a;
            }
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < n; i += kRsBlock) sidx[j0 + i] = key[i];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += kRsBlock) {
    const long o = sidx[j0 + i];
    double w[3], qi;
    int bad = 0;
    load_wrapped(xyz, q, o, g, w, &qi, &bad);
    const double rx = w[0] - cx * g.h[0], ry = w[1] - cy * g.h[1], rz = w[2] - cz * g.h[2];
    gst(spos)[j0 + i] = vec4<T>{(T)rx, (T)ry, (T)rz, (T)qi};
    if (spos64) gst(spos64)[j0 + i] = vec4<double>{rx, ry, rz, 0.0};
    gst(scx)[j0 + i] = cx;
  }
}

// FP64 pairs use the device library's erfc, exp and sqrt.
__device__ __forceinline__ double erfc_t(double x) { return erfc(x); }
__device__ __forceinline__ double exp_t(double x) { return exp(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }

// erfc(z) for z >= 0 in FP32 by the Chebyshev fit of Press et al.
// (Numerical Recipes, function erfcc; relative error below 1.2e-7):
// erfc(z) = t exp(-z^2 + P(t)), t = 1/(1 + z/2), P a degree-9 polynomial.
// gauss = exp(-z^2) is passed in (the gradient needs it as well).  Both
// exponentials use the hardware base-2 exponential (relative error ~1e-7 for
// the arguments that matter, |z| < 3; terms beyond it are below 2e-5 of the
// largest ones).
__device__ __forceinline__ float erfc_cheb(float z, float gauss) {
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.5f * z);
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  return t * gauss * __expf(p);
}

struct RsOut {
  void* phi;        // N, compute precision, or null
  void* force;      // N x 3, compute precision, or null
  double* epart;    // one energy partial per cell
  int out_grad;     // force receives grad phi instead of -q grad phi
  int accumulate;   // add into phi and force
};

// floor(a / c) for c > 0
__device__ __forceinline__ int floor_div(int a, int c) { return a >= 0 ? a / c : -((-a + c - 1) / c); }

// Pair sums of one cell's targets (one wavefront per cell).  A cell of n
// charges gives each target g = 2^k lanes (the largest with n g <= 64; g = 1
// for n > 32), which split its neighbours between them (lane sub takes every
// g-th one) and add their partial sums at the end.  Neighbours are visited by
// rows: for each (dy, dz) the cells ix - d .. ix + d that can hold a charge
// within rc (d from the row's gaps) are consecutive in the cell order, so
// their charges form one contiguous range per periodic image of x.  Of each
// chunk of 64 charges of a range only those within rc of the target cell's
// box (about two in three at two cells per cutoff) enter the pair loop,
// packed in chunk order.
//
// FP32 records round each position to a few units in the last place of the
// cell side, which is large against the difference of the closest pairs
// (and their terms, ~1/r^2, dominate the forces): a pair closer than h/8
// (a few in 10^4 of the pairs within rc) takes its difference again in FP64
// from spos64 before the pair terms are evaluated in FP32.
template <typename T, bool GRAD>
__global__ __launch_bounds__(64) void rs_sum_kernel(RsGeom g, const int* __restrict__ start,
                                                    const int* __restrict__ sidx,
                                                    const vec4<T>* __restrict__ spos,
                                                    const int* __restrict__ scx,
                                                    const vec4<double>* __restrict__ spos64, RsOut out) {
  const int cell = blockIdx.x, lane = threadIdx.x;
  const int cX = g.c[0], cY = g.c[1], cZ = g.c[2];
  const int ix = cell % cX, iy = (cell / cX) % cY, iz = cell / (cX * cY);
  const int t0 = uni(gld(start)[cell]), t1 = uni(gld(start)[cell + 1]);
  const int n = t1 - t0;
  int lg = 0;
  while (lg < 6 && (n << (lg + 1)) <= 64) ++lg;
  const int gsz = 1 << lg, per = 64 >> lg, sub = lane & (gsz - 1), tl = lane >> lg;
  const T rc2 = (T)(g.rc * g.rc), xi = (T)g.xi, xi2 = (T)(g.xi * g.xi);
  const T c2 = (T)(2.0 * g.xi / 1.7724538509055160272981674833411452);
  const double hx = g.h[0], hy = g.h[1], hz = g.h[2], rc2d = g.rc * g.rc;
  const T hxT = (T)hx, hyT = (T)hy, hzT = (T)hz;
  const double hmin = fmin(hx, fmin(hy, hz)), hmax = fmax(hx, fmax(hy, hz));
  const T near2 = (T)(hmin * hmin / 64.0);   // (h/8)^2: FP64 differences below it (FP32 records)
  // rc^2 with a margin for the rounding of records near the cell's faces
  const T box2 = (T)((g.rc * (1.0 + 1e-5) + 1e-5 * hmax) * (g.rc * (1.0 + 1e-5) + 1e-5 * hmax));
  __shared__ vec4<T> crec[64];   // kept records of the current chunk
  __shared__ int cslot[64];      // and their record slots
  double e_acc = 0.0;
  for (int tb = t0; tb < t1; tb += per) {
    const int k = tb + tl;
    const bool valid = k < t1;
    const vec4<T> tp = valid ? gld(spos)[k] : vec4<T>{(T)0, (T)0, (T)0, (T)0};
    T phi = 0, gx = 0, gy = 0, gz = 0;
    // jslot: the neighbour's record; its cell is kxb + scx[jslot], iy + ky,
    // iz + kz, unwrapped, counted from the target's cell
    auto pair = [&](T xj, T yj, T zj, T qn, bool self, int jslot, int kxb, int ky, int kz) {
      T dxv = tp.x - xj, dyv = tp.y - yj, dzv = tp.z - zj;
      T r2 = dxv * dxv + dyv * dyv + dzv * dzv;
      if (r2 < rc2 && !self) {
        if constexpr (sizeof(T) == 4) {
          if (r2 < near2 && valid) {
            const vec4<double> a = gld(spos64)[k], b = gld(spos64)[jslot];
            const double sx = (double)(gld(scx)[jslot] + kxb) * hx, sy = (double)ky * hy, sz = (double)kz * hz;
            dxv = (T)(a.x - (b.x + sx));
            dyv = (T)(a.y - (b.y + sy));
            dzv = (T)(a.z - (b.z + sz));
            r2 = dxv * dxv + dyv * dyv + dzv * dzv;
          }
        }
        T ir, e, gauss;
        if constexpr (sizeof(T) == 4) {
          ir = __builtin_amdgcn_rsqf(r2);
          gauss = __expf(-xi2 * r2);
          e = erfc_cheb(xi * r2 * ir, gauss) * ir;
        } else {
          const T r = sqrt_t(r2);
          ir = (T)1 / r;
          gauss = exp_t(-xi2 * r2);
          e = erfc_t(xi * r) * ir;
        }
        phi += qn * e;
        if constexpr (GRAD) {
          // d/dr [erfc(xi r)/r] = -erfc(xi r)/r^2 - 2 xi/sqrt(pi) exp(-xi^2 r^2)/r
          const T f = -qn * (e + c2 * gauss) * ir * ir;
          gx += f * dxv;
          gy += f * dyv;
          gz += f * dzv;
        }
      }
    };
    for (int dz = -g.s[2]; dz <= g.s[2]; ++dz) {
      const int uz = iz + dz;
      if (g.D < 3 && (uz < 0 || uz >= cZ)) continue;
      const int qz = floor_div(uz, cZ);
      const double gz_ = (double)max(0, abs(dz) - 1) * hz;
      for (int dy = -g.s[1]; dy <= g.s[1]; ++dy) {
        const int uy = iy + dy;
        if (g.D < 2 && (uy < 0 || uy >= cY)) continue;
        const int qy = floor_div(uy, cY);
        const double gy_ = (double)max(0, abs(dy) - 1) * hy;
        const double rem = rc2d - gz_ * gz_ - gy_ * gy_;
        if (rem <= 0.0) continue;
        int dm = g.s[0];   // cells in x whose gap (|dx| - 1) h_x stays below the remaining reach
        while (dm > 1 && ((dm - 1) * hx) * ((dm - 1) * hx) >= rem) --dm;
        const int rowc = ((uz - qz * cZ) * cY + (uy - qy * cY)) * cX;
        int xa = ix - dm, xb = ix + dm;
        if (g.D < 1) {
          xa = max(xa, 0);
          xb = min(xb, cX - 1);
        }
        for (int qx = floor_div(xa, cX); qx <= floor_div(xb, cX); ++qx) {
          const int lo = max(xa, qx * cX) - qx * cX, hi = min(xb, qx * cX + cX - 1) - qx * cX;
          const int j0 = uni(gld(start)[rowc + lo]), j1 = uni(gld(start)[rowc + hi + 1]);
          const bool same = qx == 0 && qy == 0 && qz == 0 && uy == iy && uz == iz;
          // neighbour positions relative to the target cell's corner: the
          // neighbour's unwrapped cell is (cx + qx c_x, iy + dy, iz + dz)
          const T oy = (T)dy * hyT, oz = (T)dz * hzT;
          const int kxb = qx * cX - ix;
          for (int jb = j0; jb < j1; jb += 64) {
            // one record per lane, moved to the target cell's frame; only the
            // records within rc of the cell's box [0, h)^3 can meet a target
            const int jn = jb + lane;
            bool keep = false;
            vec4<T> np;
            if (jn < j1) {
              np = gld(spos)[jn];
              np.x += (T)(gld(scx)[jn] + kxb) * hxT;
              np.y += oy;
              np.z += oz;
              const T ex = max(max(-np.x, np.x - hxT), (T)0), ey = max(max(-np.y, np.y - hyT), (T)0),
                      ez = max(max(-np.z, np.z - hzT), (T)0);
              keep = ex * ex + ey * ey + ez * ez < box2;
            }
            // kept records packed in chunk order into LDS, read back by every lane
            const unsigned long long m = __ballot(keep);
            const int cnt = __popcll(m);
            if (cnt == 0) continue;
            if (keep) {
              const int at = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
              crec[at] = np;
              cslot[at] = jn;
            }
            wave_sync();
            for (int u0 = 0; u0 < cnt; u0 += gsz) {
              const int u = u0 + sub;
              if (u < cnt) {
                const vec4<T> r = crec[u];
                const int js = cslot[u];
                pair(r.x, r.y, r.z, r.w, same && js == k, js, kxb, dy, dz);
              }
            }
            wave_sync();   // before the next chunk overwrites crec
          }
        }
      }
    }
    // the target's g lanes add their partial sums (fixed order)
    for (int o = 1; o < gsz; o <<= 1) {
      phi += __shfl_xor(phi, o, 64);
      if constexpr (GRAD) {
        gx += __shfl_xor(gx, o, 64);
        gy += __shfl_xor(gy, o, 64);
        gz += __shfl_xor(gz, o, 64);
      }
    }
    if (valid && sub == 0) {
      const int o = gld(sidx)[k];
      if (out.phi) {
        T* p = (T*)out.phi;
        gst(p)[o] = out.accumulate ? gld(p)[o] + phi : phi;
      }
      if (GRAD && out.force) {
        T* f = (T*)out.force;
        const T m = out.out_grad ? (T)1 : -tp.w;
        T v[3] = {m * gx, m * gy, m * gz};
#pragma unroll
        for (int d = 0; d < 3; ++d) gst(f)[3 * (long)o + d] = out.accumulate ? gld(f)[3 * (long)o + d] + v[d] : v[d];
      }
      e_acc += (double)tp.w * (double)phi;
    }
  }
  // fixed-order wavefront reduction of the cell's q phi
  for (int o = 32; o > 0; o >>= 1) e_acc += __shfl_xor(e_acc, o, 64);
  if (lane == 0 && out.epart) gst(out.epart)[cell] = e_acc;
}

// E^R = 1/2 sum_m q_m phi^R_m from the per-cell partials, in a fixed order.
__global__ __launch_bounds__(kRsBlock) void rs_energy_kernel(const double* __restrict__ epart, int ncell,
                                                             double* __restrict__ energy, int accumulate) {
  __shared__ double sh[kRsBlock];
  double v = 0.0;
  for (int i = threadIdx.x; i < ncell; i += kRsBlock) v += gld(epart)[i];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kRsBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *gst(energy) = (accumulate ? *gld(energy) : 0.0) + 0.5 * sh[0];
}

__global__ __launch_bounds__(kRsBlock) void rs_zero_kernel(int* __restrict__ p, int n) {
  const int i = blockIdx.x * kRsBlock + threadIdx.x;
  if (i < n) gst(p)[i] = 0;
}

}  // namespace
}  // namespace se

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
struct se_rs_plan {
  se::RsGeom g;
  long n_max = 0;
  bool f64 = true;
  int ncell = 0, nscan = 0;
  // workspace (caller-owned, bound by se_rs_set_workspace): byte offsets of
  // the cell counts and starts, scan sums, per-charge cells, slots and
  // sorted indices, per-cell energy partials, sorted records and (FP32 plans)
  // the records' FP64 positions
  size_t o_cnt = 0, o_start = 0, o_bsum = 0, o_cell = 0, o_slot = 0, o_sidx = 0, o_ep = 0, o_pos = 0, o_pos64 = 0;
  size_t ws_bytes = 0;
  bool ws_bound = false;
  void* mem = nullptr;  // plan-owned: the device status word
  // slot: arrival slot of each charge in its cell (bin to scatter), then the x
  // cell index of each sorted record (order to pair sums)
  int *cnt = nullptr, *start = nullptr, *bsum = nullptr, *cell_of = nullptr, *slot = nullptr, *sidx = nullptr,
      *status = nullptr;
  double* epart = nullptr;
  void* spos = nullptr;
  se::vec4<double>* spos64 = nullptr;
  size_t bytes = 0;
  // SE_PROFILE: four events per evaluation (start, pair sums start, pair
  // sums end, end), kept until se_rs_plan_profile reads them
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  double ms[3] = {0, 0, 0};
  int launches = 0;
};

namespace {
constexpr int kRsEventPool = 4 * 1024;

// smallest s with s h >= rc (rounding of rc / h taken care of)
int rs_span(double h, double rc) {
  int s = std::max(1, (int)std::ceil(rc / h));
  while (s > 1 && (s - 1) * h >= rc) --s;
  while (s * h < rc) ++s;
  return s;
}

se_status rs_plan_make(int D, const int* c, const int* sp, const double* Ls, double xi, double rc, long n_max,
                       se_precision prec, se_rs_plan** out) {
  se_rs_plan* p = new (std::nothrow) se_rs_plan();
  if (!p) return SE_ERR_NOMEM;
  p->g.D = D;
  for (int d = 0; d < 3; ++d) {
    p->g.c[d] = c[d];
    p->g.s[d] = sp[d];
    p->g.L[d] = Ls[d];
    p->g.h[d] = Ls[d] / c[d];
  }
  p->g.rc = rc;
  p->g.xi = xi;
  p->n_max = n_max;
  p->f64 = prec == SE_F64;
  p->ncell = c[0] * c[1] * c[2];
  p->nscan = (p->ncell + se::kRsScanItems - 1) / se::kRsScanItems;
  const size_t n = (size_t)std::max(1L, n_max), nc = (size_t)p->ncell;
  const size_t rec = p->f64 ? 32 : 16;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  p->o_cnt = 0;
  p->o_start = p->o_cnt + up(4 * nc);
  p->o_bsum = p->o_start + up(4 * (nc + 1));
  p->o_cell = p->o_bsum + up(4 * (size_t)p->nscan);
  p->o_slot = p->o_cell + up(4 * n);
  p->o_sidx = p->o_slot + up(4 * n);
  p->o_ep = p->o_sidx + up(4 * n);
  p->o_pos = p->o_ep + up(8 * nc);
  p->o_pos64 = p->o_pos + up(rec * n);
  p->ws_bytes = p->o_pos64 + (p->f64 ? 0 : up(32 * n));
  if (hipMalloc(&p->mem, 256) != hipSuccess) {
    delete p;
    return SE_ERR_NOMEM;
  }
  p->status = (int*)p->mem;
  p->bytes = 256;
  if (hipMemset(p->status, 0, sizeof(int)) != hipSuccess) {
    (void)hipFree(p->mem);
    delete p;
    return SE_ERR_DEVICE;
  }
  *out = p;
  return SE_OK;
}

bool rs_args_ok(int D, double xi, long n_max, se_precision prec) {
  return D >= 0 && D <= 3 && xi > 0.0 && std::isfinite(xi) && (prec == SE_F64 || prec == SE_F32) &&
         n_max <= 0x7fffffffL;
}
}  // namespace

extern "C" {

se_status se_rs_cells(double L, double rc, long n_max, int cells_per_rc, int* cells, int* span) {
  if (!cells || !span) return SE_ERR_ARG;
  if (!(L > 0.0) || !(rc > 0.0) || !std::isfinite(L) || !std::isfinite(rc) || n_max < 0) return SE_ERR_PARAM;
  const int k = cells_per_rc <= 0 ? 2 : cells_per_rc;
  if (k > 8) return SE_ERR_PARAM;
  // at most about one cell per charge, and kRsMaxCells per direction
  const int by_n = std::max(1, (int)std::floor(std::cbrt((double)std::max(1L, n_max)) + 1e-9));
  const int c = (int)std::max(1.0, std::min({std::floor(k * L / rc), (double)by_n, (double)se::kRsMaxCells}));
  *cells = c;
  *span = rs_span(L / c, rc);
  return SE_OK;
}

se_status se_rs_cells_box(const double* Ls, double rc, long n_max, int cells_per_rc, int* cells, int* span) {
  if (!Ls || !cells || !span) return SE_ERR_ARG;
  if (!(rc > 0.0) || !std::isfinite(rc) || n_max < 0) return SE_ERR_PARAM;
  for (int d = 0; d < 3; ++d)
    if (!(Ls[d] > 0.0) || !std::isfinite(Ls[d])) return SE_ERR_PARAM;
  const int k = cells_per_rc <= 0 ? 2 : cells_per_rc;
  if (k > 8) return SE_ERR_PARAM;
  // at most about one cell per charge: cells per unit length at that density
  const double V = Ls[0] * Ls[1] * Ls[2];
  if (!(V > 0.0) || !std::isfinite(V)) return SE_ERR_PARAM;
  const double per = std::cbrt((double)std::max(1L, n_max) / V);
  for (int d = 0; d < 3; ++d) {
    const double by_n = std::max(1.0, std::floor(Ls[d] * per + 1e-9));
    cells[d] = (int)std::max(1.0, std::min({std::floor(k * Ls[d] / rc), by_n, (double)se::kRsMaxCells}));
    span[d] = rs_span(Ls[d] / cells[d], rc);
  }
  return SE_OK;
}

se_status se_rs_plan_create(int D, double L, double xi, double rc, long n_max, se_precision prec,
                            int cells_per_rc, void* hip_stream, se_rs_plan** out) {
  (void)hip_stream;
  if (!out) return SE_ERR_ARG;
  *out = nullptr;
  if (!rs_args_ok(D, xi, n_max, prec)) return SE_ERR_PARAM;
  int c, s;
  const se_status st = se_rs_cells(L, rc, n_max, cells_per_rc, &c, &s);
  if (st != SE_OK) return st;
  const int c3[3] = {c, c, c}, s3[3] = {s, s, s};
  const double L3[3] = {L, L, L};
  return rs_plan_make(D, c3, s3, L3, xi, rc, n_max, prec, out);
}

se_status se_rs_plan_create_box(int D, const double* Ls, double xi, double rc, long n_max, se_precision prec,
                                int cells_per_rc, void* hip_stream, se_rs_plan** out) {
  (void)hip_stream;
  if (!out) return SE_ERR_ARG;
  *out = nullptr;
  if (!Ls) return SE_ERR_ARG;
  if (!rs_args_ok(D, xi, n_max, prec)) return SE_ERR_PARAM;
  int c3[3], s3[3];
  const se_status st = se_rs_cells_box(Ls, rc, n_max, cells_per_rc, c3, s3);
  if (st != SE_OK) return st;
  return rs_plan_make(D, c3, s3, Ls, xi, rc, n_max, prec, out);
}

se_status se_rs_workspace_size(const se_rs_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return SE_ERR_ARG;
  *bytes = plan->ws_bytes;
  return SE_OK;
}

se_status se_rs_set_workspace(se_rs_plan* p, void* ptr, size_t bytes) {
  if (!p) return SE_ERR_ARG;
  if (ptr && (((uintptr_t)ptr & 255) || bytes < p->ws_bytes)) return SE_ERR_WORKSPACE;
  char* b = (char*)ptr;
  p->ws_bound = ptr != nullptr;
  p->cnt = ptr ? (int*)(b + p->o_cnt) : nullptr;
  p->start = ptr ? (int*)(b + p->o_start) : nullptr;
  p->bsum = ptr ? (int*)(b + p->o_bsum) : nullptr;
  p->cell_of = ptr ? (int*)(b + p->o_cell) : nullptr;
  p->slot = ptr ? (int*)(b + p->o_slot) : nullptr;
  p->sidx = ptr ? (int*)(b + p->o_sidx) : nullptr;
  p->epart = ptr ? (double*)(b + p->o_ep) : nullptr;
  p->spos = ptr ? (void*)(b + p->o_pos) : nullptr;
  p->spos64 = ptr && !p->f64 ? (se::vec4<double>*)(b + p->o_pos64) : nullptr;
  return SE_OK;
}

se_status se_rs_get_info(const se_rs_plan* plan, int* cells, int* span, size_t* device_bytes) {
  if (!plan) return SE_ERR_ARG;
  if (cells) *cells = plan->g.c[0];
  if (span) *span = plan->g.s[0];
  if (device_bytes) *device_bytes = plan->bytes;
  return SE_OK;
}

se_status se_rs_get_device_status(se_rs_plan* plan, void* hip_stream) {
  if (!plan) return SE_ERR_ARG;
  int s = 0;
  if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return SE_ERR_DEVICE;
  if (hipMemcpy(&s, plan->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SE_ERR_DEVICE;
  if (s && hipMemset(plan->status, 0, sizeof(int)) != hipSuccess) return SE_ERR_DEVICE;
  if (s & 1) return SE_ERR_NONFINITE;
  if (s & 2) return SE_ERR_OUT_OF_BOX;
  return SE_OK;
}

se_status se_rs_eval(se_rs_plan* plan, long N, const void* xyz, const void* q, void* phi, void* force,
                     double* energy, unsigned flags, void* hip_stream) {
  using namespace se;
  if (!plan || N < 0 || N > plan->n_max) return SE_ERR_ARG;
  if (N > 0 && (!xyz || !q)) return SE_ERR_ARG;
  if (flags & ~(SE_IN_F32 | SE_SYNC_CHECK | SE_OUT_GRAD | SE_ACCUMULATE | SE_PROFILE)) return SE_ERR_ARG;
  if (!plan->ws_bound) return SE_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  int e0 = -1;
  if ((flags & SE_PROFILE) && N > 0) {
    if (plan->ev.empty()) {
      plan->ev.resize(kRsEventPool);
      for (auto& e : plan->ev)
        if (hipEventCreate(&e) != hipSuccess) return SE_ERR_DEVICE;
    }
    if (plan->ev_used + 4 <= (int)plan->ev.size()) e0 = plan->ev_used;   // kept once all four are recorded
  }
  auto mark = [&](int k) {
    if (e0 >= 0) (void)hipEventRecord(plan->ev[e0 + k], st);
  };
  const bool in32 = (flags & SE_IN_F32) != 0, acc = (flags & SE_ACCUMULATE) != 0;
  const int nc = plan->ncell;
  const RsGeom g = plan->g;
  if (N == 0) {
    // no charges: phi^R and its gradient are empty, the energy is zero
    if (energy && !acc) {
      rs_energy_kernel<<<1, kRsBlock, 0, st>>>(plan->epart, 0, energy, 0);   // writes 0
      if (hipGetLastError() != hipSuccess) return SE_ERR_DEVICE;
    }
    if (flags & SE_SYNC_CHECK) return se_rs_get_device_status(plan, hip_stream);
    return SE_OK;
  }
  const int nb = (int)((N + kRsBlock - 1) / kRsBlock);
  mark(0);
  rs_zero_kernel<<<(nc + kRsBlock - 1) / kRsBlock, kRsBlock, 0, st>>>(plan->cnt, nc);
  if (in32)
    rs_bin_kernel<float><<<nb, kRsBlock, 0, st>>>(g, N, (const float*)xyz, (const float*)q, plan->cnt,
                                                  plan->cell_of, plan->slot, plan->status);
  else
    rs_bin_kernel<double><<<nb, kRsBlock, 0, st>>>(g, N, (const double*)xyz, (const double*)q, plan->cnt,
                                                   plan->cell_of, plan->slot, plan->status);
  rs_scan_sums_kernel<<<plan->nscan, kRsBlock, 0, st>>>(plan->cnt, nc, plan->bsum);
  rs_scan_top_kernel<<<1, kRsBlock, 0, st>>>(plan->bsum, plan->nscan);
  rs_scan_apply_kernel<<<plan->nscan, kRsBlock, 0, st>>>(plan->cnt, nc, plan->bsum, plan->start, N);
  rs_scatter_kernel<<<nb, kRsBlock, 0, st>>>(N, plan->cell_of, plan->slot, plan->start, plan->sidx);
  const RsOut out{phi, force, plan->epart, (flags & SE_OUT_GRAD) ? 1 : 0, acc ? 1 : 0};
  if (plan->f64) {
    auto* sp = (vec4<double>*)plan->spos;
    if (in32)
      rs_order_kernel<double, float><<<nc, kRsBlock, 0, st>>>(g, (const float*)xyz, (const float*)q, plan->start,
                                                              plan->sidx, sp, plan->slot, nullptr);
    else
      rs_order_kernel<double, double><<<nc, kRsBlock, 0, st>>>(g, (const double*)xyz, (const double*)q,
                                                               plan->start, plan->sidx, sp, plan->slot, nullptr);
    mark(1);
    if (force)
      rs_sum_kernel<double, true><<<nc, 64, 0, st>>>(g, plan->start, plan->sidx, sp, plan->slot, nullptr, out);
    else
      rs_sum_kernel<double, false><<<nc, 64, 0, st>>>(g, plan->start, plan->sidx, sp, plan->slot, nullptr, out);
    mark(2);
  } else {
    auto* sp = (vec4<float>*)plan->spos;
    if (in32)
      rs_order_kernel<float, float><<<nc, kRsBlock, 0, st>>>(g, (const float*)xyz, (const float*)q, plan->start,
                                                             plan->sidx, sp, plan->slot, plan->spos64);
    else
      rs_order_kernel<float, double><<<nc, kRsBlock, 0, st>>>(g, (const double*)xyz, (const double*)q,
                                                              plan->start, plan->sidx, sp, plan->slot, plan->spos64);
    mark(1);
    if (force)
      rs_sum_kernel<float, true><<<nc, 64, 0, st>>>(g, plan->start, plan->sidx, sp, plan->slot, plan->spos64, out);
    else
      rs_sum_kernel<float, false><<<nc, 64, 0, st>>>(g, plan->start, plan->sidx, sp, plan->slot, plan->spos64, out);
    mark(2);
  }
  if (energy) rs_energy_kernel<<<1, kRsBlock, 0, st>>>(plan->epart, nc, energy, acc ? 1 : 0);
  mark(3);
  if (hipGetLastError() != hipSuccess) return SE_ERR_DEVICE;
  if (e0 >= 0) plan->ev_used += 4;
  if (flags & SE_SYNC_CHECK) return se_rs_get_device_status(plan, hip_stream);
  return SE_OK;
}

se_status se_rs_plan_profile(se_rs_plan* plan, void* hip_stream, se_stage_record* out, int cap, int* n,
                             int reset) {
  if (!plan || !n || (cap > 0 && !out)) return SE_ERR_ARG;
  if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return SE_ERR_DEVICE;
  for (int e = 0; e + 4 <= plan->ev_used; e += 4) {
    float t[3];
    for (int k = 0; k < 3; ++k)
      if (hipEventElapsedTime(&t[k], plan->ev[e + k], plan->ev[e + k + 1]) != hipSuccess) return SE_ERR_DEVICE;
    for (int k = 0; k < 3; ++k) plan->ms[k] += t[k];
    ++plan->launches;
  }
  plan->ev_used = 0;
  static const char* const names[3] = {"rs_cells", "rs_pairs", "rs_energy"};
  *n = 0;
  for (int k = 0; k < 3 && *n < cap; ++k) {
    se_stage_record& r = out[(*n)++];
    std::memset(&r, 0, sizeof(r));
    std::snprintf(r.name, sizeof(r.name), "%s", names[k]);
    r.launches = plan->launches;
    r.ms_total = plan->ms[k];
  }
  if (reset) {
    plan->ms[0] = plan->ms[1] = plan->ms[2] = 0.0;
    plan->launches = 0;
  }
  return SE_OK;
}

se_status se_rs_plan_destroy(se_rs_plan* plan) {
  if (!plan) return SE_OK;
  for (auto& e : plan->ev) (void)hipEventDestroy(e);
  if (plan->mem) (void)hipFree(plan->mem);
  delete plan;
  return SE_OK;
}

}  // extern "C"
