// Internal declarations shared by the host planner (se_plan.cpp) and the
// gfx950 kernels (se_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace se {

constexpr int kMaxStages = 16;
constexpr int kMaxClasses = 3;
constexpr int kMaxP = 16;
constexpr int kMaxNu = 12;
constexpr int kBlock = 256;      // threads per block (transforms and gathering: below)
// Gathering stages a (T + P - 1)^3 grid region per tile, so few of its
// workgroups fit a CU; eight wavefronts per workgroup keep more region loads
// in flight.
constexpr int kGatherBlock = 512;
constexpr int kMaxBlock = kGatherBlock;
constexpr int kSB = 4;           // sub-bin edge in grid cells (particle sort key)
constexpr int kMaxOwnRanges = 256;  // sub-bin rows of one tile ((T/kSB)^2 <= 256 for T <= 64)
// Clipped spreading: most anchor pieces (periodic images) per direction and
// most particle ranges per tile.
constexpr int kMaxPieces = 4;
// Particle records one gather workgroup holds in LDS at a time.
constexpr int kGatherBatch = 256;
// Column spreading: particles per weight batch, and most tile points per column.
constexpr int kColBatch = 128;
constexpr int kColZ = 16;
constexpr int kMaxClipRanges = 512;
// Most periodic images of tile boxes one fold block sums over in a direction.
constexpr int kMaxFoldImages = 8;
// Most samples (transform length x pencils) one FFT workgroup holds, and the
// FFT workgroup size.
constexpr int kFftCap = 8192;
constexpr int kFftBlock = 256;
// LDS budget of an FFT workgroup: the transforms are latency bound, so a pass
// takes fewer pencils per workgroup rather than fewer workgroups per CU (four
// per 160 KB CU at this budget).  Across a batch the largest pass sets every
// system's occupancy.
constexpr size_t kFftLdsSoft = 40 * 1024;
// Passes whose blocks hold at most this many samples (transform length x
// pencils) run their stages in place in one LDS buffer (inputs of a stage
// held in registers); passes with a larger samples cap alternate between two
// buffers.
constexpr int kFftInplaceCap = 2048;
// Butterflies of radix R one thread holds in registers across an in-place
// stage: enough for kFftInplaceCap samples at every radix (R = 3 holds 3,
// R = 5 and 7 hold 2); the planner keeps (n / R) F <= kFftIpIters(R)
// kFftBlock at every stage (F complex transforms per block).
constexpr int kFftIpIters(int R) {
  return R == 7 ? 2 : (R == 5 ? 2 : (R == 3 ? 3 : (kFftInplaceCap + R * kFftBlock - 1) / (R * kFftBlock)));
}

// Green's-function modes of the fused scaling pass (Eq. scale).
enum GMode : int {
  G_NONE = 0,
  G_INVSQ = 1,  // 1/|k|^2 from squared-wavenumber tables; 0 where |k| = 0 (Eq. G_hat_3d)
  G_TAB1 = 2,   // table over the pencil coordinate t (2P zero mode, Eq. G_hat_2d)
  G_TAB2 = 3,   // folded table over (b0, t) (1P zero mode, Eq. G_hat_1d)
  G_TAB3 = 4    // folded table over (b0, b1, t) (0P, Algorithm 3 output)
};

// K_FUSED_D: the fused pass of force method 2 (Section 7.2), whose scaling
// carries the factor i k_d of one direction d (FftPass::deriv); single plans
// only (batch transform lists hold kinds 0..4).
enum FftKind : int { K_C2C_FWD = 0, K_C2C_INV = 1, K_R2C = 2, K_C2R = 3, K_FUSED = 4, K_FUSED_D = 5 };

// One group of pencils that share a transform length.  A pencil is addressed
// by (b0, b1); its sample t sits at base + b0*s0 + b1*s1 + t*st (in complex
// elements, or real elements for real input/output).
struct FftClass {
  int n, n_in, n_out;
  int nst;
  int rad[kMaxStages];
  unsigned long long radpack;     // rad[] packed 4 bits per stage, stage 0 lowest
  const void* in;
  void* out;
  const void* tw;                 // twiddles exp(-2 pi i k/n), k < n, in the compute precision
  long long in_st, in_s0, in_s1;
  long long out_st, out_s0, out_s1;
  // scaling of the fused pass: S = sA[b0+offA] sB[b1+offB] sC[t] G
  int gmode;
  int offA, offB;
  const void* sA;
  const void* sB;
  const void* sC;
  const void* kA;
  const void* kB;
  const void* kC;
  const void* gtab;
  int gd0, gd1;                   // table extents of the b0 (fastest) and b1 indices:
                                  // G_TAB2 [t][b0], G_TAB3 [t][b1][b0]
  int fold1, fold2;               // transform lengths used to fold b1 and t
  int fold0;                      // transform length used to fold b0 (0: b0 not folded)
  // force method 2: signed wavenumbers k of the b0 (A), b1 (B) and pencil (C)
  // directions, indexed as sA, sB, sC (0 at the Nyquist index of an even
  // length), and the physical directions (0 x, 1 y, 2 z) of A and B; the
  // pencil direction of a fused pass is z
  const void* dA;
  const void* dB;
  const void* dC;
  int dirA, dirB;
};

struct FftPass {
  FftClass cls[kMaxClasses];
  const int4* items;              // per block: {class, b0_start, b1, count}
  int nitems;
  int B;                          // pencils per block (even for the paired real passes when > 1)
  int nmax;                       // largest n (LDS sizing)
  int kind;
  int xcd;                        // item mapping: 0 plain, 1 one range per XCD, c >= 2 chunks of c
  int wide;                       // 1 if a workgroup's pencils span 4 GiB or more (64-bit offsets)
  int inplace;                    // 1: stages in place in one LDS buffer
  int deriv;                      // K_FUSED_D: direction d of the factor i k_d
  double alg_bytes, alg_flops;    // algorithmic counts of one launch (tracing only)
};

// Geometry and window of the gridding / gathering kernels.
struct GridGeom {
  int D;
  int G[3];           // grid points per direction (x, y, z)
  int per[3];         // 1 if the direction is periodic
  int d0[3];          // integer offset of the free-direction grid origin, (Mt - M)/2
  int T[3];           // tile edges in grid points (multiples of kSB)
  int nt[3];          // tiles per direction
  int nsb[3];         // sub-bins per direction, ceil(G / kSB)
  int chunk;          // particles per wavefront round of the spread kernel (<= 64)
  int xcd;            // tile mapping: 0 plain, 1 one range per XCD, c >= 2 chunks of c
  int clip;           // spreading: 0 boxes + fold, 1 clipped stencils, 2 columns (both write the grid)
  int P, nu;
  int window;         // 0 Gaussian, 1 PKB
  double h, L, xi;
  double Lp[3];       // box side per periodic direction (L, or M_d h in a rectangular 3P box)
  double alpha;       // Gaussian shape
  double scale;       // 4 pi h^3 (trapezoidal rule of Eq. complete_integral)
};

// Device buffers of one evaluation.
struct EvalBuffers {
  int* sb_count;      // sub-bins
  int* sb_start;      // sub-bins + 1
  int* sb_cursor;     // sub-bins
  int* p_key;         // n_max: sub-bin of each particle (input order)
  int* p_cell;        // n_max: packed cell of each particle (input order)
  void* p_frac;       // n_max x 4 (fx, fy, fz, q) in compute precision (input order)
  int* s_cell;        // n_max: sorted packed cells
  int* s_idx;         // n_max: sorted original indices
  void* s_fq;         // n_max x 4 sorted (fx, fy, fz, q)
  int* bsum;          // per scan block: count total
  void* stage;        // per tile: spread box (T+P-1)^3 in compute precision
  double* qpart;      // per bin block: sum q, sum |q|, sum q^2
  double* epart;      // per gather block: sum q phi
  double* red;        // 4 doubles: Q, sum|q|, Q2, E
  int* status;        // device status word
  const void* wtab;   // window coefficient table (compute precision)
  void* grid;         // real grid G[0]*G[1]*G[2]
  void* vjp_phi;      // n_max: A g of an adjoint evaluation (compute precision)
  void* vjp_grad;     // n_max x 3: grad (A g) of an adjoint evaluation
};

// One system of a batch: its geometry, buffers and transform passes, and
// where its particles sit in the concatenated input/output arrays.
constexpr int kPasses = 5;
struct SysDesc {
  GridGeom g;
  EvalBuffers b;
  FftPass pass[kPasses];
  long long N;        // particles of the system
  long long off;      // index of its first particle in the concatenated arrays
  int nblk_bin;       // bin / scatter work items
  int nscan;          // scan work items
  int ntiles;         // spread / fold / gather work items
  int check_neutral;  // D >= 1
  double self_coef;   // -2 xi / sqrt(pi)
};

// Inputs and outputs of a batched evaluation (concatenated over systems).
struct BatchIO {
  const void* xyz;
  const void* q;
  void* phi;
  void* force;
  double* energy;     // one per system
  int in_f32, out_grad, add_self, allow_nonneutral;
  int xcd_tiles, xcd_fft;   // item mapping modes of the tile / transform stages (as GridGeom::xcd)
  int fft_wide;             // bit k: transform stage k needs 64-bit offsets for some system
  const int4* fft_rec;      // work records of the transform lists, concatenated in list order
};

// Stages of a batched evaluation, in order; one launch per stage.
enum BatchStage : int {
  BS_ZERO = 0, BS_BIN, BS_SCAN1, BS_SCAN2, BS_SCATTER, BS_ORDER, BS_SPREAD, BS_FOLD,
  BS_FFT0, BS_FFT1, BS_FFT2, BS_FFT3, BS_FFT4, BS_GATHER, BS_ENERGY, BS_COUNT
};
constexpr int stage_block(int st) {
  return st >= BS_FFT0 && st <= BS_FFT4 ? kFftBlock : (st == BS_GATHER ? kGatherBlock : kBlock);
}
// Work lists of a batch: one per stage, and for the transform stages one per
// (stage, transform kind) so that each launch runs a single kind.
constexpr int kFftKinds = 5;
constexpr int BL_COUNT = BS_COUNT + 5 * kFftKinds;
constexpr int fft_list(int st, int kind) { return BS_COUNT + (st - BS_FFT0) * kFftKinds + kind; }

// Launchers (se_kernels.hip).  All enqueue on 'st' and return the HIP error.
hipError_t launch_bin(const GridGeom& g, const EvalBuffers& b, long N, const void* xyz,
                      const void* q, bool in_f32, bool f64, int nblk, hipStream_t st);
hipError_t launch_scan(const GridGeom& g, const EvalBuffers& b, int nblk_bin, int check_neutral,
                       hipStream_t st);
hipError_t launch_scatter(const GridGeom& g, const EvalBuffers& b, long N, bool f64, hipStream_t st);
hipError_t launch_order(const GridGeom& g, const EvalBuffers& b, int nsbtot, bool f64, hipStream_t st);
hipError_t launch_spread(const GridGeom& g, const EvalBuffers& b, bool f64, hipStream_t st);
hipError_t launch_fold(const GridGeom& g, const EvalBuffers& b, bool f64, hipStream_t st);
// Gathering modes: GM_ALL phi and grad phi (Eq. force-method-1, forces by
// method 1) and the per-tile energy partials; GM_PHI phi and the energy
// partials only; GM_COMP one force component by method 2: 'force' column
// comp receives -q (or 1 with out_grad) times the gathered value of a grid
// that holds the derivative along comp.
enum GatherMode : int { GM_ALL = 0, GM_PHI = 1, GM_COMP = 2 };
hipError_t launch_gather(const GridGeom& g, const EvalBuffers& b, bool f64, void* phi, void* force,
                         int out_grad, double self_coef, hipStream_t st, int mode = GM_ALL, int comp = 0);
hipError_t launch_energy(const GridGeom& g, const EvalBuffers& b, double* energy, double self_e,
                         hipStream_t st);
// Sub-bin counts set to zero (a fill kernel, so that the evaluation records
// no memset node when a caller captures it in a graph).
hipError_t launch_zero(const GridGeom& g, const EvalBuffers& b, hipStream_t st);
// Adjoint combinations of the autograd layer (FP64 arithmetic, outputs in the
// input precision in_f32 ? float : double; phi, grad, ag, agrad in the compute
// precision f64 ? double : float).  Either output may be null.
//   energy:    gx = gE q grad,  gq = gE phi                 (gE: device scalar)
//   potential: gx = g grad + q agrad,  gq = ag
hipError_t launch_energy_vjp(long N, bool in_f32, bool f64, const double* gE, const void* q, const void* phi,
                             const void* grad, void* gx, void* gq, hipStream_t st);
hipError_t launch_potential_vjp(long N, bool in_f32, bool f64, const void* q, const void* g, const void* grad,
                                const void* ag, const void* agrad, void* gx, void* gq, hipStream_t st);
// Transforms (se_fft.hip).
hipError_t launch_fft(const FftPass& p, bool f64, hipStream_t st);
size_t fft_lds_bytes(const FftPass& p, bool f64);
// One transform kind of transform stage 'pass' of a batch: 'nitems' work
// records {system * 4 + class, b0 start, b1, count} at 'rec' (device).
void launch_batch_fft(bool f64, int kind, bool wide, const SysDesc* sys, const int4* rec, int pass, int nitems,
                      size_t lds, int xcd, hipStream_t st);
size_t spread_lds_bytes(const GridGeom& g, bool f64);
size_t gather_lds_bytes(const GridGeom& g, bool f64);
int scan_blocks(const GridGeom& g);

// Batched evaluation: one launch per stage over the work items of all systems.
// off: device table [BL_COUNT][nsys + 1] of work-item prefix sums per work
// list; items: host array of the list totals; lds: dynamic LDS bytes per stage;
// ev: BS_COUNT + 1 events recorded before each stage and after the last, or null.
hipError_t launch_batch(int P, bool f64, const SysDesc* sys, int nsys, const int* off, const int* items,
                        const BatchIO& io, const size_t* lds, hipStream_t st, hipEvent_t* ev);

// 0P precompute helpers (FP64).
hipError_t launch_g0p_fill(double* buf, int n0, double h, double R, hipStream_t st);
hipError_t launch_g0p_truncate(const double* big, int n0, double* small, int Mt, hipStream_t st);
hipError_t launch_g0p_fold(const double* full, int Mt, void* table, bool f64, hipStream_t st);

}  // namespace se
