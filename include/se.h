/*
 * se.h -- C ABI of the MI355X Spectral Ewald k-space library.
 *
 * The library computes the Fourier-space (k-space) part of the electrostatic
 * potential of N point charges with periodicity D in {3,2,1,0}, by the
 * Spectral Ewald method of Shamshirgar, Bagge and Tornberg, "Fast Ewald
 * summation for electrostatic potentials with arbitrary periodicity"
 * (arXiv:1712.04732):
 *
 *   problem      Section 2, Eq. (potential): charges q_n at x_n in [0,L)^3,
 *                lattice P_D of periodic images; the k-space part is
 *                Eq. (fourier_space_nonzero_ewald), the self term Section 2.
 *   method       Algorithm 4 (gridding, FFT / adaptive FFT (Algorithm 1) /
 *                zero-padded FFT, scaling by Eq. (scale) with the modified
 *                Green's functions of Section 3.1, IFFT / AIFT (Algorithm 2),
 *                gathering by the trapezoidal rule of Eq. (complete_integral)).
 *   precompute   Algorithm 3 (free space), done once per plan in FP64.
 *   windows      Section 4: truncated Gaussian, Eq. (gaussian); KB window
 *                Eq. (kaiser_window) evaluated as the piecewise polynomial
 *                (PKB) of Section 4.1.
 *   parameters   Section 6 (Table lambda, Eqs. estimate-s, estimate-nl).
 *   forces       Section 7.2, method 1, Eq. (force-method-1).
 *
 * Conventions shared by every entry point
 *   - Device pointers are HIP device addresses on the device current when the
 *     plan was created.  Host pointers are marked "host".
 *   - Positions: N x 3, row-major (x0,y0,z0,x1,...).  Periodic directions are
 *     the first D coordinates (x; x,y; x,y,z).  Periodic coordinates may lie
 *     anywhere (they are wrapped into [0,L)); free coordinates must lie in
 *     [0,L).
 *   - Position and charge arrays are float64, or float32 when the flag
 *     SE_IN_F32 is given.  Potentials and gradients are written in the plan's
 *     compute precision (se_params.prec).  Energies are always float64.
 *   - All work is enqueued on the HIP stream passed in (NULL = the default
 *     stream) and returns without waiting, except where SE_SYNC_CHECK is set.
 *   - Ownership: the caller owns every input and output buffer and the
 *     workspace, one block of device memory per plan that holds all work
 *     buffers of an evaluation (sorted particles, grid, spectra, partial
 *     sums); se_plan_workspace_size reports its size and
 *     se_plan_set_workspace binds it (batches and real-space plans likewise).
 *     A plan itself owns only its tables (window coefficients, twiddles,
 *     scaling vectors, Green's-function tables, transform work lists) and its
 *     device status word.  Nothing is allocated or freed during an
 *     evaluation.
 *   - No exceptions cross the ABI; every call returns an se_status.
 */
#ifndef SE_MI355X_H
#define SE_MI355X_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SE_OK = 0,
  SE_ERR_ARG = 1,         /* NULL pointer, negative size, bad flag combination   */
  SE_ERR_PARAM = 2,       /* parameters violate Section 3.3 / Section 6 rules    */
  SE_ERR_NONNEUTRAL = 3,  /* |sum q| > 1e-10 sum |q| for D = 1, 2, 3 (Section 2) */
  SE_ERR_OUT_OF_BOX = 4,  /* a free-direction coordinate outside [0, L)           */
  SE_ERR_NONFINITE = 5,   /* NaN or Inf in positions or charges                   */
  SE_ERR_DEVICE = 6,      /* a HIP runtime call failed                            */
  SE_ERR_NOMEM = 7,       /* device allocation failed in se_plan_create           */
  SE_ERR_UNSUPPORTED = 8, /* valid request this build does not implement           */
  SE_ERR_WORKSPACE = 9    /* no workspace bound, or one too small or misaligned     */
} se_status;

/* Windows of Section 4: truncated Gaussian (Eq. gaussian), the KB window
 * evaluated as the piecewise polynomial of Section 4.1 (PKB), and the
 * exponential of semicircle (ES, Eq. expsemicirc_window), evaluated directly,
 * whose Fourier transform the planner computes by quadrature. */
typedef enum { SE_WIN_GAUSSIAN = 0, SE_WIN_PKB = 1, SE_WIN_ES = 2 } se_window;
typedef enum { SE_F64 = 0, SE_F32 = 1 } se_precision;

/* Parameters of one system (Algorithm 4 input list, Section 6 rules).
 * Fields marked "<= 0 -> default" take the paper's rule when left at 0. */
typedef struct {
  int D;              /* periodic directions: 3, 2, 1 or 0                       */
  double L;           /* box side along x (the cube's side), > 0                 */
  double xi;          /* Ewald parameter xi > 0 (Eq. gamma)                      */
  int M;              /* grid intervals per periodic side, even, 7-smooth        */
  int P;              /* window support in grid intervals, even, 2..16, P <= M   */
  se_window window;
  double shape;       /* alpha (Gaussian) / beta (KB, ES); <= 0 -> (pi/2) P 0.91 /
                         2.5 P (both KB and ES)                                  */
  int nu;             /* PKB polynomial degree; <= 0 -> min(P/2 + 2, 9)          */
  double lambda;      /* free-direction extension factor; <= 0 -> Table lambda
                         (the ES window takes the KB values)                     */
  double s0;          /* zero-mode / free-space upsampling; <= 0 -> 2 / 2.5 / 2.8 */
  double s;           /* AFT upsampling of the set I (Eq. I); <= 0 -> Eq. estimate-s */
  int n_l;            /* size of the set I; < 0 -> Eq. estimate-nl                */
  double tol;         /* absolute rms tolerance for the s, n_l estimates          */
  double Q;           /* sum of q^2, used by the s, n_l estimates (B, Section 5.2) */
  se_precision prec;  /* compute precision of grid, FFT, gather                   */
  int tile;           /* cubic spread/gather tile edge (multiple of 4); <= 0 -> automatic */
  int tile3[3];       /* spread/gather tile edges x, y, z (multiples of 4, each <= 32);
                         all > 0 -> used instead of 'tile'                          */
  int fft_cap;        /* samples (length x pencils) per FFT workgroup: a power of two
                         in 1024..8192; <= 0 -> 2048 (FP32) / 1024 (FP64); up to
                         2048 the stages run in place in one LDS buffer, above it
                         they alternate between two                                */
  int xcd_tiles;      /* workgroup -> tile mapping of spread, fold and gather (the
                         8 XCDs take workgroups in turn): < 0 plain order, 1 one
                         contiguous tile range per XCD, c >= 2 chunks of c
                         neighbouring tiles per XCD, 0 -> 1                        */
  int xcd_fft;        /* the same for the transform passes' pencil groups            */
  int spread_mode;    /* 1: each tile spreads its particles' whole stencils into an
                         LDS box with halo, boxes are summed by a fold pass;
                         2: each tile adds the parts of all stencils that reach it
                         and writes the grid directly (no staging, no fold);
                         3: as 2, but each thread sums the stencils covering its
                         own grid column in registers (no atomics; tiles with
                         x*y <= 256 and z <= 16);
                         0 -> 3 below 0.1 particles per grid point, else 1        */
  int force_method;   /* forces and grad phi (Section 7.2): 0 or 1 method 1, the
                         gradient of the gathering window (Eq. force-method-1);
                         2 method 2, the scaling step times i k_d and steps 4-5
                         once per direction d, each gathering with the window
                         itself (single plans only)                            */
  int deriv_fit;      /* PKB, method 1: 0 differentiates the PKB polynomial (the
                         exact gradient of the discrete energy); 1 fits W'_KB
                         by its own polynomial with the same P, beta, nu
                         (Section 7.2; the gradient is then not the energy's
                         exact derivative)                                      */
  int My, Mz;         /* rectangular periodic cells (Section 2 notes that the
                         domain need not be a cube): grid intervals along y
                         and z at the same spacing h = L/M, so a triply
                         periodic box is L x My h x Mz h and a doubly periodic
                         cell L x My h (z free, extent L, Mz = M); even,
                         7-smooth, >= P; <= 0 -> M.  D = 3 (My, Mz) or D = 2
                         (My only); SE_ERR_PARAM otherwise                      */
} se_params;

/* Derived sizes of a plan (read-only report). */
typedef struct {
  int D, M, P, nu;
  int Mt;             /* extended free-direction grid, Section 3.3 (rounded, see below) */
  int n0;             /* length of the zero-mode (2P/1P) or precompute (0P) transform  */
  int nI;             /* length of the set-I transforms (2P/1P)                        */
  int n_l;            /* size of the set I                                             */
  int grid[3];        /* gridding grid points in x, y, z                               */
  int nfft[3];        /* transform lengths of the periodic / 0P padded directions      */
  int tile[3];        /* spread/gather tile edges in grid points (x, y, z)             */
  int fft_cap;        /* samples per FFT workgroup in use                              */
  int spread_mode;    /* spreading mode in use (1 boxes and fold, 2 clipped, 3 columns) */
  int fft_wide;       /* bit k: transform pass k addresses with 64-bit offsets (its
                         workgroups' pencils span 4 GiB or more)                    */
  double h, shape, lambda, s0, s, R;
  size_t device_bytes; /* device memory held by the plan (tables, status word)         */
  size_t workspace_bytes; /* workspace an evaluation needs (se_plan_workspace_size)    */
  int fft_block[5];   /* pencils per transform workgroup of each pass (real pencils,
                         two per complex transform, for the real-to-complex and
                         complex-to-real passes); 0 for a pass the plan lacks   */
} se_plan_info;

typedef struct se_plan se_plan;

/* eval flags */
#define SE_IN_F32      0x1u  /* positions and charges are float32               */
#define SE_ADD_SELF    0x2u  /* add phi_self = -2 xi/sqrt(pi) q (Section 2)     */
#define SE_SYNC_CHECK  0x4u  /* wait for the stream and report device-side errors */
#define SE_OUT_GRAD    0x8u  /* 'force' receives grad phi instead of -q grad phi */
#define SE_ALLOW_NONNEUTRAL 0x10u /* skip the neutrality check (adjoint passes whose
                                     'charges' are cotangents)                     */
#define SE_PROFILE     0x20u  /* record a HIP event pair around every kernel launch */
#define SE_ACCUMULATE  0x40u  /* se_rs_eval: add into phi, force and energy       */

/* Fill *out with the paper's parameter rules (Section 6) for a system of N
 * charges with sum of squares Q: shape, nu, lambda, s0, and s, n_l from the
 * absolute tolerance tol (Eqs. estimate-s, estimate-nl).  M and P are taken
 * as given (the grid and support that the caller chose).
 * Errors: SE_ERR_ARG for out == NULL; SE_ERR_PARAM for invalid D, L, xi,
 * M, P or tol. */
se_status se_params_default(int D, double L, double xi, int M, int P, se_window window,
                            double Q, double tol, se_precision prec, se_params* out);

/* The parameter recipe of Section 6 for a relative tolerance tol_rel (an
 * absolute rms tolerance tol_rel * B, B = sqrt(Q) f_c(xi L)/L of Section 5.2)
 * at a given xi and window support P: M is the smallest even 7-smooth grid
 * size whose Kolafa-Perram k-space estimate, Eq. (KP_fourier_space), meets the
 * tolerance and for which P <= f_W(M/(xi L)) (no error pollution, Eq.
 * error_pollution); the other fields as se_params_default.
 * Errors: SE_ERR_ARG for out == NULL; SE_ERR_PARAM for invalid inputs or when
 * no M below 4096 qualifies. */
se_status se_params_for_tolerance(int D, double L, double xi, double Q, double tol_rel, int P,
                                  se_window window, se_precision prec, se_params* out);

/* The whole parameter selection of Section 6 for a relative tolerance tol_rel
 * (absolute rms tolerance eps = tol_rel * B) at a given xi: the grid
 * M = 2 k_inf of Eq. (KP_kinf) (the inverse of the k-space estimate, by the
 * Lambert W function), rounded up to an even integer with prime factors 2,
 * 3, 5, 7 only; the window support P from the approximation estimates
 * eps = 2 B e^{-(pi/2) P c} (Gaussian) or 10 B e^{-2.5 P} (PKB), rounded up
 * to an even integer; when P > f_W(M/(xi L)) (error pollution, Eq.
 * error_pollution) M is increased by 5 % and P by 4; then the rules of
 * se_params_default (shape, nu, lambda, s0, s, n_l).
 * Errors: SE_ERR_ARG for out == NULL; SE_ERR_PARAM for invalid inputs or a
 * result beyond the supported sizes (P > 16, M >= 4096). */
se_status se_params_recipe(int D, double L, double xi, double Q, double tol_rel, se_window window,
                           se_precision prec, se_params* out);

/* The error scale of Section 5.2, B = sqrt(Q) f_c(xi L) / L with f_c of
 * Eq. (fc-expression) and Q = sum of q^2: relative tolerances of the other
 * calls are tolerances on rms errors divided by B.  *B receives it (host).
 * Errors: SE_ERR_ARG for B == NULL; SE_ERR_PARAM for Q < 0, xi <= 0, L <= 0
 * or non-finite inputs. */
se_status se_error_scale(double Q, double xi, double L, double* B);

/* Real-space cutoff for a relative tolerance tol_rel (absolute rms tolerance
 * tol_rel * B): Eq. (KP_rc), the inverse of the Kolafa-Perram real-space
 * estimate Eq. (KP_real_space), by the principal branch of the Lambert W
 * function.  *rc receives the cutoff (host).
 * Errors: SE_ERR_ARG for rc == NULL; SE_ERR_PARAM for non-positive or
 * non-finite L, xi, Q, tol_rel. */
se_status se_rs_cutoff_for_tolerance(double L, double xi, double Q, double tol_rel, double* rc);

/* Validate the parameters (Section 3.3 and 3.4: lambda >= 1, s >= 1 and
 * s0 >= 1 + sqrt(3 - D) for D < 3), derive the grids (Section 3.3: Mt = 2
 * ceil((M + lambda P)/2); Mt, s0 Mt and s Mt are rounded up to even integers
 * with prime factors 2, 3, 5, 7 only), build the FP64 tables (PKB coefficients by the
 * Vandermonde solve of Eq. polynomial-linsys, separable scaling vectors of
 * Eq. scale, Green's-function tables of Eqs. G_hat_0d..G_hat_3d), allocate
 * device memory for up to n_max particles, and for D = 0 run Algorithm 3 on
 * the GPU in FP64.  hip_stream: the hipStream_t used for the setup work.
 * On success *out owns device memory until se_plan_destroy.
 * Errors: SE_ERR_ARG, SE_ERR_PARAM, SE_ERR_NOMEM, SE_ERR_DEVICE. */
se_status se_plan_create(const se_params* params, long n_max, void* hip_stream, se_plan** out);

/* Copy the derived sizes of a plan into *info (host). */
se_status se_plan_get_info(const se_plan* plan, se_plan_info* info);

/* Bytes of device workspace one evaluation of the plan needs (host output):
 * the work buffers of Algorithm 4 for n_max particles (binned and sorted
 * particle records, the gridding grid, the spectra of the transform passes,
 * block partial sums, and the buffers of se_eval_vjp).
 * Errors: SE_ERR_ARG for NULL arguments. */
se_status se_plan_workspace_size(const se_plan* plan, size_t* bytes);

/* Bind a caller-owned workspace: ptr is a device address aligned to 256
 * bytes with at least se_plan_workspace_size bytes, owned by the caller (for
 * example a torch tensor) and kept alive while evaluations that use it may
 * run.  Every later se_eval / se_eval_vjp uses it; its contents need no
 * initialisation and are overwritten by each evaluation, so evaluations that
 * share one workspace must be ordered (one stream).  ptr = NULL unbinds.
 * No device work is enqueued.
 * Errors: SE_ERR_ARG (plan NULL); SE_ERR_WORKSPACE (misaligned or too small). */
se_status se_plan_set_workspace(se_plan* plan, void* ptr, size_t bytes);

/* One evaluation of Algorithm 4 for N <= n_max charges.
 *   xyz    device, N x 3 positions (float64, or float32 with SE_IN_F32)
 *   q      device, N charges (same dtype as xyz)
 *   phi    device, N potentials phi~^{D,F} (+ phi_self with SE_ADD_SELF), or NULL
 *   force  device, N x 3 forces -q grad phi (Eq. force-method-1, gradient of the
 *          gathering window), or grad phi with SE_OUT_GRAD, or NULL
 *   energy device, one float64: E = 1/2 sum_m q_m phi_m (+ the self energy
 *          -xi/sqrt(pi) sum q^2 with SE_ADD_SELF), or NULL
 * The energy is one half of the paper's E^F = sum q phi (Section 7.2): with the
 * half, dE/dq = phi and -dE/dx = the forces above.
 * Errors: SE_ERR_ARG (bad pointers, N > n_max); SE_ERR_WORKSPACE (no
 * workspace bound); with SE_SYNC_CHECK also SE_ERR_NONFINITE,
 * SE_ERR_OUT_OF_BOX, SE_ERR_NONNEUTRAL, SE_ERR_DEVICE.
 * Without SE_SYNC_CHECK device-side errors are latched and reported by
 * se_get_device_status; outputs of such a call are not meaningful. */
se_status se_eval(se_plan* plan, long N, const void* xyz, const void* q, void* phi, void* force,
                  double* energy, unsigned flags, void* hip_stream);

/* Size of the library's static scratch array (see se_eval_static). */
#define SE_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* se_eval for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Arguments, outputs and errors as se_eval; the plan's workspace binding is
 * neither needed nor changed.  The work buffers lie in a static device array
 * of SE_STATIC_SCRATCH_BYTES (128 MiB) that the library holds on each device
 * it runs on until the process ends; nothing is allocated or freed.  The
 * array keeps the last call's contents, and each evaluation clears what it
 * accumulates itself.  Every call on one device shares that device's array:
 * calls that overlap on one device (two streams, two threads) race and give
 * undefined results, so they must be ordered by the caller.  The current
 * device must be the plan's device.
 * Errors: as se_eval; SE_ERR_WORKSPACE when the plan's workspace
 * (se_plan_workspace_size) exceeds SE_STATIC_SCRATCH_BYTES; SE_ERR_ARG also
 * for SE_PROFILE (its event pool would be created on first use). */
se_status se_eval_static(se_plan* plan, long N, const void* xyz, const void* q, void* phi, void* force,
                         double* energy, unsigned flags, void* hip_stream);

/* Adjoint of phi = A(x) q (the vector-Jacobian product of the potential).
 * The discrete operator A of Algorithm 4 (gridding, scaling, gathering with
 * the same window) is symmetric, so for a cotangent g of phi:
 *   grad_q   = A g  (+ phi_self(g) = -2 xi/sqrt(pi) g with SE_ADD_SELF)
 *   grad_x_m = g_m grad phi(x_m) + q_m grad(A g)(x_m)   (Eq. force-method-1)
 * The library runs Algorithm 4 with the charges g (no neutrality check) and
 * combines the results in FP64.
 *   xyz, q, g   device, N x 3 / N / N, float64 (float32 with SE_IN_F32)
 *   grad_phi    device, N x 3 in the plan's precision: grad phi of the
 *               forward evaluation (se_eval with SE_OUT_GRAD); may be NULL
 *               when grad_x is NULL
 *   grad_x      device, N x 3 in the input precision, or NULL
 *   grad_q      device, N in the input precision, or NULL
 * Flags: SE_IN_F32, SE_ADD_SELF, SE_SYNC_CHECK.  Uses the bound workspace.
 * Errors: as se_eval. */
se_status se_eval_vjp(se_plan* plan, long N, const void* xyz, const void* q, const void* g, const void* grad_phi,
                      void* grad_x, void* grad_q, unsigned flags, void* hip_stream);

/* Adjoint of the energy E = 1/2 sum_m q_m phi_m of se_eval (or of se_eval
 * plus se_rs_eval with SE_ACCUMULATE): with dE/dq = phi and
 * dE/dx_m = q_m grad phi(x_m) (Section 7.2), for a cotangent grad_E of E
 *   grad_x = grad_E q grad_phi,   grad_q = grad_E phi   (FP64 arithmetic).
 *   grad_E      device, one float64
 *   q           device, N, float64 (float32 with SE_IN_F32)
 *   phi         device, N in precision prec, or NULL when grad_q is NULL
 *   grad_phi    device, N x 3 in precision prec, or NULL when grad_x is NULL
 *   grad_x      device, N x 3 in the input precision, or NULL
 *   grad_q      device, N in the input precision, or NULL
 * Flags: SE_IN_F32.  Enqueued on hip_stream; no plan or workspace needed.
 * Errors: SE_ERR_ARG, SE_ERR_DEVICE. */
se_status se_energy_vjp(long N, se_precision prec, const double* grad_E, const void* q, const void* phi,
                        const void* grad_phi, void* grad_x, void* grad_q, unsigned flags, void* hip_stream);

/* Wait for the stream, then report (and clear) the device-side status word of
 * the plan's last evaluations. */
se_status se_get_device_status(se_plan* plan, void* hip_stream);

/* Per-launch timing record (tracing subsystem).  bytes and flops are the
 * algorithmic counts of one launch: each array element the step must read or
 * write counted once, and the arithmetic of the step itself (window weights,
 * stencil sums, 5 n log2 n per length-n complex transform). */
typedef struct {
  char name[32];
  int launches;       /* launches accumulated since the last reset            */
  double ms_total;    /* summed duration from HIP events on the eval stream   */
  double bytes;       /* algorithmic bytes per launch                         */
  double flops;       /* algorithmic flops per launch                         */
} se_stage_record;

/* Wait for the stream, then aggregate the event pairs recorded by every
 * se_eval call with SE_PROFILE since the last reset into at most 'cap'
 * records (host array 'out'), one per launch site; *n receives the count.
 * reset != 0 drops the recorded events afterwards.  The event pool holds
 * 4096 pairs; launches beyond it are not recorded.
 * Errors: SE_ERR_ARG, SE_ERR_DEVICE. */
se_status se_plan_profile(se_plan* plan, void* hip_stream, se_stage_record* out, int cap, int* n,
                          int reset);

/* Release all device memory of the plan.  NULL is accepted. */
se_status se_plan_destroy(se_plan* plan);

/* ---- Batched evaluation: many independent systems, one launch per stage ----
 * Each system s has its own parameters params[s] (any D, L, xi, M) and N[s]
 * charges; all systems share P (4, 6, 8, 10 or 12), the window and the
 * precision.  Positions, charges, potentials and forces of all systems are
 * concatenated in system order (system s starts at sum_{r<s} N[r]).  One
 * evaluation runs Algorithm 4 for every system: each stage of the path (bin,
 * scan, scatter, spread, fold, five transform passes, gather, energy) is one
 * launch whose workgroups are the work items (particle blocks, tiles, pencil
 * groups) of all systems, so the whole batch costs 14 launches.
 * Errors: SE_ERR_ARG; SE_ERR_UNSUPPORTED when P, window or precision differ
 * between systems, P is not instantiated for batches or a system asks for
 * force method 2; SE_ERR_PARAM,
 * SE_ERR_NOMEM, SE_ERR_DEVICE as se_plan_create. */
typedef struct se_batch_plan se_batch_plan;

se_status se_batch_plan_create(const se_params* params, const long* N, int n_sys, void* hip_stream,
                               se_batch_plan** out);

/* Derived sizes of system 'sys' (host outputs, each may be NULL);
 * *reserved receives 0 (the output is reserved). */
se_status se_batch_plan_get_info(const se_batch_plan* plan, int sys, se_plan_info* info,
                                 long* n_particles, int* reserved);

/* Workspace of a batch: the workspaces of its systems one after another.
 * Arguments and errors as se_plan_workspace_size / se_plan_set_workspace;
 * binding uploads the systems' descriptors (synchronous host-to-device copy),
 * so it must not overlap an evaluation of the same batch plan. */
se_status se_batch_plan_workspace_size(const se_batch_plan* plan, size_t* bytes);
se_status se_batch_plan_set_workspace(se_batch_plan* plan, void* ptr, size_t bytes);

/* One batched evaluation.  xyz, q: device, concatenated as above (float64, or
 * float32 with SE_IN_F32); phi (sum N), force (sum N x 3): device, compute
 * precision, or NULL; energy: device, n_sys float64 energies, or NULL.  Flags
 * as for se_eval (SE_PROFILE records an event before each stage launch). */
se_status se_eval_batch(se_batch_plan* plan, const void* xyz, const void* q, void* phi, void* force,
                        double* energy, unsigned flags, void* hip_stream);

/* Wait for the stream, then report the SE_PROFILE batched evaluations since
 * the last reset: one record per stage launch that has work (zero, bin, scan1,
 * scan2, scatter, spread, fold, fft0..fft4, gather, energy), timed with HIP
 * events between the stage launches, then one record "batch_all_stages" for
 * the whole evaluation; at most 'cap' records into host 'out', count in *n.
 * bytes and flops are the algorithmic counts of one launch, summed over the
 * systems.  reset != 0 clears the accumulated times.
 * Errors: SE_ERR_ARG, SE_ERR_DEVICE. */
se_status se_batch_plan_profile(se_batch_plan* plan, void* hip_stream, se_stage_record* out, int cap, int* n,
                                int reset);

/* Wait for the stream, report and clear the device status of every system
 * (the most severe code wins). */
se_status se_batch_get_device_status(se_batch_plan* plan, void* hip_stream);

/* Release the batch plan and its sub-plans.  NULL is accepted. */
se_status se_batch_plan_destroy(se_batch_plan* plan);

/* ---- autotuner ---------------------------------------------------------
 * Schedule knobs (tile3, fft_cap, xcd_tiles, xcd_fft) chosen by timing
 * candidate plans on the caller's own input with HIP events: first the tile
 * shape of spread / fold / gather (their summed time), then the FFT samples
 * per workgroup (the transform passes' time), then the XCD mappings.  The
 * result is kept only if the whole evaluation is faster than with the
 * default knobs.  The numbers computed by a tuned plan are those of the
 * default plan up to rounding (the method's parameters are not touched). */
typedef struct {
  int candidates;      /* settings timed                                          */
  double ms_default;   /* one evaluation with the default knobs (sum of launches) */
  double ms_tuned;     /* one evaluation with the chosen knobs                    */
} se_tune_report;

/* Tune one system.  params: the plan parameters (method fields as for
 * se_plan_create); xyz, q: device input of N >= 1 particles (float64, or
 * float32 with flags SE_IN_F32; SE_ALLOW_NONNEUTRAL accepted); tuned: host,
 * receives params with the knobs set; report: host or NULL.  Allocates
 * temporary output buffers and creates and destroys one plan per candidate
 * on 'hip_stream'; the stream is synchronised.
 * Errors: SE_ERR_ARG, SE_ERR_NOMEM, SE_ERR_UNSUPPORTED (no candidate ran). */
se_status se_autotune(const se_params* params, long N, const void* xyz, const void* q, unsigned flags,
                      void* hip_stream, se_params* tuned, se_tune_report* report);

/* Tune a batch (arguments as for se_batch_plan_create and se_eval_batch):
 * tile shape and FFT samples per workgroup are chosen for each periodicity
 * class on that class's systems, then one XCD mapping for the whole batch.
 * tuned: host array of n_sys params. */
se_status se_batch_autotune(const se_params* params, const long* N, int n_sys, const void* xyz, const void* q,
                            unsigned flags, void* hip_stream, se_params* tuned, se_tune_report* report);

/* ---- Real-space part on the GPU ----------------------------------------
 * The short-range sum of the Ewald split, Eq. (real_space_ewald):
 *   phi^R_m = sum_{p in P_D} sum_n' q_n erfc(xi r) / r,  r = |x_m - x_n + p|,
 * over the pairs with r < rc (the prime drops n = m at p = 0), and its
 * gradient.  Together with se_eval (SE_ADD_SELF) it gives the full potential
 * phi = phi^R + phi^F + phi^self of Eq. (potential_split); the error of the
 * cutoff is bounded by Eq. (KP_real_space) of Section 5.2.
 * Positions and charges follow the conventions above (periodic coordinates
 * wrapped, free ones in [0, L)).  A cell list of c^3 cells with c <= cells_per_rc
 * L / rc serves the pair search; charges are ordered by cell and, inside a
 * cell of at most 2048 charges, by input index, so results repeat bit for
 * bit from run to run. */
typedef struct se_rs_plan se_rs_plan;

/* Cells per direction and neighbour span (host only, no device work):
 * c = max(1, min(floor(cells_per_rc L / rc), floor(cbrt(n_max)), 160)) and the
 * smallest s with s L / c >= rc, so every pair within rc lies in the
 * (2s+1)^3 cells around a charge's cell.  cells_per_rc <= 0 means 2.
 * Errors: SE_ERR_ARG for NULL outputs; SE_ERR_PARAM for L, rc not positive
 * and finite, n_max < 0 or cells_per_rc > 8. */
se_status se_rs_cells(double L, double rc, long n_max, int cells_per_rc, int* cells, int* span);

/* A real-space plan for up to n_max charges of periodicity D in a box of side
 * L with Ewald parameter xi and cutoff rc, sums in precision prec.  The plan
 * owns only its device status word; the work buffers of an evaluation (cell
 * counts and offsets, sorted records, energy partials) lie in a caller-owned
 * workspace (se_rs_workspace_size, se_rs_set_workspace).
 * Errors: SE_ERR_ARG (out NULL), SE_ERR_PARAM (D, xi, prec, n_max > 2^31-1,
 * or as se_rs_cells), SE_ERR_NOMEM. */
se_status se_rs_plan_create(int D, double L, double xi, double rc, long n_max, se_precision prec,
                            int cells_per_rc, void* hip_stream, se_rs_plan** out);

/* Cells and spans of a triply periodic rectangular box of sides Ls[0] x
 * Ls[1] x Ls[2] (Section 2: the box need not be a cube), host only.  Per
 * direction d: c_d = max(1, min(floor(cells_per_rc Ls[d] / rc),
 * floor(Ls[d] cbrt(n_max / V)), 160)) with V the box volume (about one cell
 * per charge at most), and the smallest s_d with s_d Ls[d] / c_d >= rc.
 * Ls: host, 3 values; cells, span: host, 3 values each.
 * Errors: SE_ERR_ARG for NULL pointers; SE_ERR_PARAM for a side or rc not
 * positive and finite, n_max < 0 or cells_per_rc > 8. */
se_status se_rs_cells_box(const double* Ls, double rc, long n_max, int cells_per_rc, int* cells, int* span);

/* As se_rs_plan_create for periodicity D in a rectangular box of sides
 * Ls[0] x Ls[1] x Ls[2] (host, 3 values): periodic coordinates wrapped by
 * their direction's side, free ones in [0, Ls[d]); cells of
 * se_rs_cells_box.  The rectangular cells of a se_params with M, My, Mz grid
 * intervals at spacing h = L / M are Ls = {L, My h, Mz h} (D = 3) and
 * Ls = {L, My h, L} (D = 2, z free).  se_rs_get_info reports the x direction.
 * Errors: SE_ERR_ARG (Ls or out NULL), SE_ERR_PARAM (D, xi, prec, n_max, or
 * as se_rs_cells_box), SE_ERR_NOMEM. */
se_status se_rs_plan_create_box(int D, const double* Ls, double xi, double rc, long n_max, se_precision prec,
                                int cells_per_rc, void* hip_stream, se_rs_plan** out);

/* Workspace of a real-space plan: size in bytes (host output), and binding
 * of a caller-owned block (device, 256-byte aligned, at least that size;
 * NULL unbinds).  As se_plan_workspace_size / se_plan_set_workspace.
 * Errors: SE_ERR_ARG (NULL plan or output); SE_ERR_WORKSPACE. */
se_status se_rs_workspace_size(const se_rs_plan* plan, size_t* bytes);
se_status se_rs_set_workspace(se_rs_plan* plan, void* ptr, size_t bytes);

/* Cells per direction, span and plan-owned device bytes of a plan (host
 * outputs, each may be NULL).  Errors: SE_ERR_ARG for plan NULL. */
se_status se_rs_get_info(const se_rs_plan* plan, int* cells, int* span, size_t* device_bytes);

/* One evaluation for N <= n_max charges.
 *   xyz, q  device, as for se_eval (float64, or float32 with SE_IN_F32)
 *   phi     device, N values phi^R in the plan's precision, or NULL
 *   force   device, N x 3: -q grad phi^R, or grad phi^R with SE_OUT_GRAD, or NULL
 *   energy  device, one float64: E^R = 1/2 sum_m q_m phi^R_m, or NULL
 * With SE_ACCUMULATE the results are added to what phi, force and energy
 * hold (for example the output of se_eval on the same charges).  N = 0 writes
 * a zero energy (or leaves it with SE_ACCUMULATE).
 * Flags: SE_IN_F32, SE_OUT_GRAD, SE_ACCUMULATE, SE_SYNC_CHECK, SE_PROFILE.
 * Errors: SE_ERR_ARG (pointers, N, flags); SE_ERR_WORKSPACE (none bound);
 * with SE_SYNC_CHECK also
 * SE_ERR_NONFINITE, SE_ERR_OUT_OF_BOX and SE_ERR_DEVICE. */
se_status se_rs_eval(se_rs_plan* plan, long N, const void* xyz, const void* q, void* phi, void* force,
                     double* energy, unsigned flags, void* hip_stream);

/* Wait for the stream, then report and clear the plan's device status word. */
se_status se_rs_get_device_status(se_rs_plan* plan, void* hip_stream);

/* Wait for the stream, then report the se_rs_eval calls made with SE_PROFILE
 * since the last reset (a pool of 1024 calls; later ones are not recorded):
 * three records, "rs_cells" (binning, scan, scatter and ordering by cell),
 * "rs_pairs" (the pair sums) and "rs_energy", with the summed HIP-event time
 * and the number of calls; bytes and flops are left 0 (the pair count
 * depends on the input).  At most 'cap' records into host 'out', count in
 * *n; reset != 0 clears the sums.  Errors: SE_ERR_ARG, SE_ERR_DEVICE. */
se_status se_rs_plan_profile(se_rs_plan* plan, void* hip_stream, se_stage_record* out, int cap, int* n,
                             int reset);

/* Release the plan's device memory.  NULL is accepted. */
se_status se_rs_plan_destroy(se_rs_plan* plan);

/* Static English text of a status code. */
const char* se_status_string(se_status s);

#ifdef __cplusplus
}
#endif

#endif /* SE_MI355X_H */
