/*
 * scarff.h - C ABI of the MI355X (gfx950) Cartesian form-factor engine.
 *
 * The engine evaluates the transition form factor of a molecule in a
 * contracted Cartesian Gaussian basis,
 *
 *     f_s(q) = s_f * sum_{mu,nu} T^s_{mu nu} <phi_mu| e^{i q.r} |phi_nu>,
 *
 * for a batch of transitions s (paper Sec. 2.2, the form-factor definition
 * with AO-basis transition density matrices; Sec. 4, eq. CartesianMethod
 * for the separable closed form that is evaluated).  The spin factor s_f is
 * 1 by default; the paper's sqrt(2) for singlet spin degeneracy (Sec. 2.2)
 * is set with scff_set_options.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units: bohr for positions, bohr^-2 for exponents, atomic units for q.
 *  - Shells: l = 0, 1, 2 (s, p, Cartesian d).  Component order inside a
 *    shell is s; x, y, z; xx, xy, xz, yy, yz, zz.  AO index mu runs over
 *    shells in the order given, components fastest.  T is given in that
 *    order.
 *  - Ownership: the caller owns every buffer.  Loads copy their inputs; no
 *    caller pointer is retained after a call returns.
 *  - Errors: every int-returning call returns SCFF_OK (0) or a negative
 *    code; scff_last_error() then describes the failure.  A failed call
 *    leaves the context as it was and writes no output, with one exception:
 *    scff_load_molecule failing while it copies the new tables to the
 *    device (out of memory or budget) leaves no molecule loaded.
 *  - Threading: a context is not re-entrant; use one context per thread or
 *    serialise calls.  The server (scff_server_*) is thread-safe.
 *  - Device: one context drives one HIP device.  Device output pointers
 *    must be device memory of that device (e.g. from torch.empty(...,
 *    device='cuda')); the call is then asynchronous on the given stream.
 *    Successive calls on one context may use different streams: each call's
 *    device work is ordered after the context's previous asynchronous work.
 */
#ifndef SCARFF_H
#define SCARFF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define SCFF_OK          0
#define SCFF_EINVAL     -1   /* malformed argument (shape, range, NULL)         */
#define SCFF_ENOMEM     -2   /* allocation failed or HBM budget exceeded       */
#define SCFF_EDEVICE    -3   /* no usable HIP device / a HIP call failed        */
#define SCFF_ESTATE     -4   /* call out of order (e.g. eval before loads)      */
#define SCFF_EBUSY      -5   /* server queue full / ticket not finished         */
#define SCFF_ECANCELLED -6   /* server request cancelled                        */

/* ---- precision of the pair contraction (paper Sec. 5.3 step "final grid
 *      contraction"; precision is this engine's choice) -------------------- */
#define SCFF_FP32    0   /* FP32 generator + FP32 MFMA contraction              */
#define SCFF_BF16X3  1   /* FP32 generator + split-BF16 (hi*hi+hi*lo+lo*hi) MFMA */

typedef struct scff_ctx scff_ctx;

/* q_a = linspace(qmin[a], qmax[a], n[a]) on each axis a (endpoints included);
 * n[a] == 1 gives the single value qmin[a].  Output element order is
 * [state][ix][iy][iz] with iz fastest. */
typedef struct {
    int n[3];
    double qmin[3];
    double qmax[3];
} scff_grid;

typedef struct {
    int nbf;                          /* Cartesian basis functions            */
    int n_shells;
    int n_states;
    long long shell_pairs_total;      /* unique shell pairs A <= B            */
    long long pairs_total;            /* unique component pairs mu <= nu      */
    long long pairs_kept;             /* K: component pairs after screening   */
    long long prim_pairs_total;       /* sum over component pairs of prim pairs */
    long long prim_comp_pairs_kept;   /* R: (component pair, prim pair) terms kept */
    size_t device_bytes;              /* device memory held by the context    */
    long long work_units;             /* units of 8 packed (virtual) pairs    */
    long long work_chunks;            /* staging steps of the grid kernel per
                                         tile: runs of 1-4 units, <= 72 terms */
} scff_info;

/* Version string of the library, static storage. */
const char* scff_version(void);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next call on this thread. */
const char* scff_last_error(void);

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the
 * device memory the context may hold (0 = no cap); exceeding it fails with
 * SCFF_ENOMEM.  Returns SCFF_EDEVICE if no HIP device is usable. */
int scff_create(int device, size_t hbm_budget_bytes, scff_ctx** out);

/* Release every resource of the context (NULL is ignored).  Waits for the
 * context's own outstanding device work (e.g. an evaluation into device
 * outputs still running on a caller stream) before freeing its buffers;
 * other contexts' work is not waited for.  A context may instead be kept
 * and reused for another molecule: it keeps every device buffer that is
 * large enough for the next problem. */
void scff_destroy(scff_ctx* ctx);

/*
 * Load geometry and basis (paper Sec. 5.1 "hierarchical data structure";
 * App. A for the primitive form and its normalisation).
 *   xyz_bohr     [n_atoms*3]     atom positions
 *   shell_atom   [n_shells]      atom index of each shell
 *   shell_l      [n_shells]      0, 1 or 2
 *   shell_nprim  [n_shells]      primitives per shell (1..32)
 *   exps, coefs  [sum nprim]     exponents alpha_k > 0 (bohr^-2) and
 *                                contraction coefficients d_k, concatenated
 *                                in shell order
 *   normalise    1: every primitive is scaled to unit self-overlap and every
 *                contracted Cartesian component to unit norm; 0: primitives
 *                are unit-normalised, the d_k are used as given.
 *   nbf_out      (may be NULL) number of Cartesian basis functions.
 * Invalidates previously loaded transitions if nbf changes.  Invalid input is
 * rejected before any device state changes (SCFF_EINVAL); if copying the
 * tables to the device fails (SCFF_ENOMEM, SCFF_EDEVICE) the previous
 * molecule is gone as well and the context has no molecule loaded.
 */
int scff_load_molecule(scff_ctx* ctx, int n_atoms, const double* xyz_bohr, int n_shells,
                       const int* shell_atom, const int* shell_l, const int* shell_nprim,
                       const double* exps, const double* coefs, int normalise, int* nbf_out);

/*
 * Load the AO-basis transition density matrices (paper Sec. 2.2, T_pq).
 *   T  [n_states][nbf][nbf] row-major, real.  1 <= n_states <= 32.
 * Only (T + T^T)/2 contributes (Omega_{mu nu} = Omega_{nu mu}); the engine
 * packs T_{mu nu} + T_{nu mu} per unique pair.
 */
int scff_load_transitions(scff_ctx* ctx, int n_states, const double* T);

/*
 * Same as scff_load_transitions with T already in device memory of the
 * context's device: T_dev [n_states][nbf][nbf] FP64, copied on hip_stream
 * (asynchronous; the caller keeps T_dev valid until the stream reaches the
 * copy).  Later calls on this context, on any stream, are ordered after
 * the copy.  T_dev is not checked for non-finite entries.
 */
int scff_load_transitions_device(scff_ctx* ctx, int n_states, const double* T_dev, void* hip_stream);

/*
 * Options.  screen_eps >= 0: pair screening threshold (paper Sec. 5.3,
 * thresholding of Cartesian pair terms).  A (component pair, primitive pair)
 * term is dropped only if, for every transition, the dropped terms' summed
 * q-independent magnitude bounds stay below screen_eps times the sum of all
 * term bounds of that transition.  0 disables screening.
 * spin_factor multiplies every result (default 1.0; sqrt(2) gives the
 * paper's singlet normalisation).
 */
int scff_set_options(scff_ctx* ctx, double screen_eps, double spin_factor);

/*
 * Evaluate on a Cartesian q-grid (paper Sec. 5.3, full-grid materialisation
 * of eq. CartesianMethod).
 *   precision      SCFF_FP32 or SCFF_BF16X3
 *   f              complex64 interleaved [n_states][nx][ny][nz][2], or NULL
 *   f2             |f|^2 float [n_states][nx][ny][nz], or NULL
 *   out_on_device  1: f/f2 are device pointers, the call is asynchronous on
 *                  hip_stream (NULL = default stream); 0: host pointers, the
 *                  call returns when they are filled.
 *   hip_stream     a hipStream_t of the context's device, or NULL.
 * Requires a loaded molecule and transitions (else SCFF_ESTATE).
 * Grid sizes: 1 <= n[a] <= 4096.
 * Device memory: the context keeps its 1D tables, host-output staging and,
 * for grids whose tile count would leave launch rounds partly idle, an FP64
 * buffer of split pair sums (at most 1 GiB) between calls.  A split that the
 * context's HBM budget cannot hold is not taken (the grid is evaluated
 * unsplit, equal up to the order of the FP64 sums).
 */
int scff_eval_grid(scff_ctx* ctx, const scff_grid* grid, int precision, float* f, float* f2,
                   int out_on_device, void* hip_stream);

/*
 * Allocation-free variant of scff_eval_grid, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  It computes exactly what
 * scff_eval_grid computes into device outputs, with the same kernels, but
 * calls no hipMalloc, hipFree or allocating library routine: the 1D tables
 * of the grid, and the FP64 partial sums of a split chunk list when they
 * fit after the tables, live in a static per-device scratch array of
 * 256 MiB (held by every device the library runs on until the process ends;
 * the 190-function, 64^3 problem's tables take 81 MB).
 *   f, f2          device pointers as for scff_eval_grid with
 *                  out_on_device = 1 (either may be NULL); asynchronous on
 *                  hip_stream (NULL = default stream).
 * Requires the precompute of the loaded problem to have run: after the
 * last scff_load_*, scff_set_options call, call scff_query or an
 * evaluation once (else SCFF_ESTATE; the precompute allocates).  A grid
 * whose 1D tables exceed the scratch (rows x (roundup16(max n) + 16) x 8
 * bytes > 256 MiB) is rejected with SCFF_EINVAL before any device work; a
 * split whose partial sums do not fit is not taken (the grid is evaluated
 * unsplit, equal up to the order of the FP64 sums).  Every call on one GPU
 * shares that GPU's scratch, which keeps the last call's contents (every
 * value a call reads is written by that call first): calls that overlap on
 * one GPU (other streams, other contexts, other threads) race and must be
 * serialised by the caller.
 */
int scff_eval_grid_noalloc(scff_ctx* ctx, const scff_grid* grid, int precision, float* f, float* f2,
                           void* hip_stream);

/*
 * Symmetric-grid mode (off by default).  The transition densities are real,
 * so f(-q) = f(q)* (Sec. 4: e^{iq.r} is the only complex factor of the
 * integrand).  With enable = 1, scff_eval_grid on a grid symmetric about
 * q = 0 (qmin[a] == -qmax[a] on every axis of n[a] > 1 points, and
 * qmin[a] == 0 on every one-point axis) evaluates the planes ix < ceil(nx/2)
 * and writes every other point as the conjugate of its mirror point
 * (nx-1-ix, ny-1-iy, nz-1-iz); |f|^2 is copied.  Other grids are evaluated
 * in full.  enable must be 0 or 1 (else SCFF_EINVAL).
 */
int scff_set_symmetry(scff_ctx* ctx, int enable);

/*
 * Evaluate at arbitrary points q [n_q][3] (host array, a.u.; paper Sec. 5.3:
 * individual points from the V-tensors).  Same outputs as scff_eval_grid
 * with the grid axes replaced by the point index: f [n_states][n_q][2],
 * f2 [n_states][n_q].  1 <= n_q <= 2^24.  precision must be SCFF_FP32 (the
 * points kernel runs on the FP32 vector units, with the same FP32 block
 * sums folded into FP64 every 32 pairs as the grid kernel's FP32 path);
 * SCFF_BF16X3 is rejected with SCFF_EINVAL.  The call waits for its
 * stream: it returns with the outputs written (host or device pointers).
 */
int scff_eval_points(scff_ctx* ctx, int n_q, const double* q, int precision, float* f,
                     float* f2, int out_on_device, void* hip_stream);

/*
 * Per-kernel timing.  With enable = 1 the context records HIP events (on the
 * stream of the call) around the pair precompute, the 1D-table kernel and
 * the fused grid kernel of each evaluation; scff_last_timing waits for the
 * last evaluation's events and reports those durations in milliseconds
 * (prep_ms is 0 when that evaluation reused an existing precompute).  Off
 * by default.  Any pointer may be NULL.
 */
int scff_set_timing(scff_ctx* ctx, int enable);
int scff_last_timing(scff_ctx* ctx, float* prep_ms, float* vtable_ms, float* grid_ms);

/* Sizes and screening statistics of the loaded problem. */
int scff_query(scff_ctx* ctx, scff_info* info);

/*
 * One-dimensional V-tensors of the loaded molecule on a grid (paper Sec. 5.3,
 * the option to compute only the 1D V-tensors, eq. CartesianVector).  For
 * every kept (component pair, primitive pair) term t and axis a the engine
 * holds V_t^a(q_a) on the grid axis; f_s(q) = sum_t Tp_s(t) V_t^x V_t^y V_t^z.
 * Writes, as host arrays:
 *   n_terms_out            R (number of kept terms)
 *   vx, vy, vz             complex64 [R][n_a][2] (NULL to skip an axis)
 *   tp                     float [n_states][R]: the packed, normalised
 *                          transition weights (NULL to skip)
 * Call first with all array pointers NULL to learn R.
 */
int scff_export_vtensors(scff_ctx* ctx, const scff_grid* grid, long long* n_terms_out, float* vx,
                         float* vy, float* vz, float* tp);

/*
 * The FFT method (paper Sec. 3, eqs. PhiTDM, Falbega, continuFFT, fftABC,
 * qabc; Sec. 5.2; the Parseval check of Sec. 7).  The transition density
 *     Phi_s(r) = s_f sum_{mu nu} T^s_{mu nu} phi_mu(r) phi_nu(r)
 * is tabulated on the periodic real-space grid
 *     x_a = xmin[a] + i_a L[a] / n[a],  i_a = 0 .. n[a]-1,
 * and Fourier transformed; the result approximates f_s at
 *     q_a = 2 pi (j_a - n[a]/2) / L[a],  j_a = 0 .. n[a]-1
 * (most negative frequency first) as
 *     f_s(q) = V_pix sum_r Phi_s(r) e^{+i q.r},  V_pix = prod_a L[a] / n[a],
 * which converges to the exact form factor as the box grows and the spacing
 * shrinks (the method's discretisation is the caller's choice: the paper
 * takes x_lim = pi / dq and dx = 2 pi / q_lim).
 *   grid       n[a] powers of two in 1..1024; L[a] > 0 (bohr)
 *   precision  SCFF_FP32 or SCFF_BF16X3: the arithmetic of the density
 *              contraction (below)
 *   f          complex64 [n_states][n0][n1][n2] interleaved, or NULL
 *   f2         |f|^2, float [n_states][n0][n1][n2], or NULL
 *   phi        the transition density Phi_s, float [n_states][n0][n1][n2], or NULL
 *   parseval   host double [n_states][2]: (sum_r |Phi_s|^2 V_pix,
 *              sum_q |f_s|^2 dq^3 / (2 pi)^3), equal by Parseval's identity
 *              up to rounding; or NULL
 * f, f2 and phi are host buffers (out_on_device = 0, the call returns when
 * they are written) or device buffers (out_on_device = 1, asynchronous on
 * hip_stream unless parseval is requested, which waits for the stream).
 * The density is FP32 (AO values built in FP64 and rounded once, weights
 * contracted on the matrix cores with FP64 sums over each 16 functions;
 * SCFF_BF16X3 splits weights and AO values into BF16 hi + lo halves and
 * keeps hi*hi + hi*lo + lo*hi, about 2^-16 relative per product, in half
 * the matrix-core instructions),
 * the transform FP32 radix-2, the corner phase FP64.  The context's
 * screening threshold is not applied (primitives below the FP32 range are
 * skipped); the spin factor is.  Basis size: up to 1232 functions.
 * SCFF_EINVAL for bad sizes, no output or a basis too large, SCFF_ESTATE
 * before a molecule and transitions are loaded, SCFF_ENOMEM over the budget.
 */
typedef struct {
    int n[3];
    double xmin[3];   /* corner of the box, bohr */
    double L[3];      /* box lengths, bohr */
} scff_fft_grid;

int scff_eval_fft(scff_ctx* ctx, const scff_fft_grid* grid, int precision, float* f, float* f2, float* phi,
                  double* parseval, int out_on_device, void* hip_stream);

/* With scff_set_timing(ctx, 1): HIP-event durations (ms) of the last
 * scff_eval_fft's weight packing, transition-density kernel, and transforms
 * with the finishing kernel (and the Parseval sums); waits for them.
 * SCFF_ESTATE if no timed FFT evaluation was recorded. */
int scff_last_fft_timing(scff_ctx* ctx, float* pack_ms, float* density_ms, float* transform_ms);

/*
 * The spherical method (paper Sec. 4 eqs. DTensor, WTensor, YYY,
 * SphericalMethod, RTensor; Sec. 5.4; App. B): the form factor on spheres of
 * radius q (a.u.) expanded in complex spherical harmonics (Condon-Shortley
 * phase, orthonormal),
 *     f_s(q, theta, phi) = sum_{l <= lmax} sum_{m} R^s_lm(q) Y_l^m(theta, phi),
 * where R^s_lm(q) = int dOmega Y_l^m* f_s is computed exactly (up to rounding,
 * in FP64) from the pair precompute: per Gaussian centre of a primitive pair
 * the monomial coefficients are turned into harmonics, the plane wave
 * e^{i q.P} is expanded in spherical Bessel functions and harmonics, and the
 * two are coupled with Gaunt coefficients.  The truncation at lmax is the
 * method's only approximation (it converges quickly, see the paper's figure
 * of the angular average); the screening threshold is not applied.
 *   lmax       0..48
 *   q          n_q radii (host array, >= 0), n_q in 1..4096
 *   n_theta, n_phi
 *              the angular grid theta_i = pi i / (n_theta - 1),
 *              phi_j = 2 pi j / n_phi (n_theta >= 2 when f or f2 is requested)
 *   R          complex128 [n_states][n_q][(lmax+1)^2][2], index l^2 + l + m, or NULL
 *   f, f2      complex64 [n_states][n_q][n_theta][n_phi][2] and float
 *              [n_states][n_q][n_theta][n_phi], or NULL
 *   avg        <|f_s|^2>_Omega(q) = sum_lm |R^s_lm(q)|^2 / (4 pi), double
 *              [n_states][n_q], or NULL
 * Outputs are host (out_on_device = 0) or device buffers (1); the call
 * returns when they are written.  SCFF_EINVAL for bad sizes or no output,
 * SCFF_ESTATE before a molecule and transitions are loaded, SCFF_ENOMEM over
 * the budget.  Device memory held by the context: the per-geometry tables
 * (harmonics to L = lmax + 4 and the W tensor, 16 bytes per geometry and
 * entry), the Bessel table of every radius, and a workspace for the row
 * operands of a batch of radii (n_states x 25 x geometries x 16 bytes per
 * radius, at most 4 GiB or an eighth of a set HBM budget, at least one
 * radius).
 */
int scff_eval_spherical(scff_ctx* ctx, int lmax, int n_q, const double* q, int n_theta, int n_phi, double* R,
                        float* f, float* f2, double* avg, int out_on_device, void* hip_stream);

/* With scff_set_timing(ctx, 1): HIP-event durations (ms) of the last
 * scff_eval_spherical's geometry kernel (W tensor and harmonics of the
 * centres), contraction over geometries, and the rest (Gaunt coupling,
 * angular average, angular grid); waits for them.  SCFF_ESTATE if no timed
 * spherical evaluation was recorded. */
int scff_last_sph_timing(scff_ctx* ctx, float* geom_ms, float* contraction_ms, float* rest_ms);

/*
 * Separable integral (paper Sec. 5.3: integrals of the form
 * I = int d^3q f(q_x) g(q_y) h(q_z) f_S(q), evaluated from the 1D V-tensors
 * with a cost linear in the axis sizes instead of their product):
 *     out_s = sum_{ix,iy,iz} wx[ix] wy[iy] wz[iz] f_s(q_ix, q_iy, q_iz)
 *           = sum_t Tp_s(t) (sum_ix wx[ix] V^x_t(q_ix)) (sum_iy ...) (sum_iz ...)
 * on the grid's axes (q_a = linspace(qmin[a], qmax[a], n[a])).  The caller
 * folds its functions and quadrature weights into the weights (e.g. f(q_x)
 * times a trapezoid weight).
 *   wx, wy, wz   complex128 interleaved [n[a]][2], host arrays
 *   out          complex128 [n_states][2], host array
 * Everything runs in FP64 on the device (rows, products, FP64 transition
 * weights), with the context's screening and spin factor; the call returns
 * when out is written.  SCFF_EINVAL for NULL or non-finite arguments,
 * SCFF_ESTATE before a molecule and transitions are loaded.
 */
int scff_eval_separable(scff_ctx* ctx, const scff_grid* grid, const double* wx, const double* wy,
                        const double* wz, double* out);

/*
 * Low-momentum limit (paper Sec. 6, oscillator-strength reconstruction):
 * f_s(q) = f_s(0) + i q . mu_s + O(q^2) with the transition dipole
 * mu_s = grad_q Im f_s at q = 0 (= s_f sum T_{mu nu} <phi_mu| r |phi_nu>).
 * mu_s is evaluated exactly from the 1D V-tensor rows' values and first
 * derivatives at q = 0, in FP64.  With the transition energies dE (a.u.),
 * f0_s = (2/3) dE_s |mu_s|^2 (atomic units, m_e = 1).
 *   dE   [n_states] host, or NULL (then f0 must be NULL)
 *   mu   [n_states][3] host, required
 *   f0   [n_states] host, or NULL
 */
int scff_dipole(scff_ctx* ctx, const double* dE, double* mu, double* f0);

/*
 * The paper's fit form of the same limit (Sec. 6): the angular average
 * <|f_s(q)|^2>_Omega on 8 shells |q| = q_fit k / 8 (k = 1..8), each averaged
 * with the product rule of 6 Gauss-Legendre nodes in cos(theta) and 12
 * equally spaced azimuths (exact for polynomials of degree < 12 on the
 * sphere), |f|^2 evaluated on the device in FP64; then the least-squares fit
 * <|f|^2> = A + B q^2 + C q^4, whose B = |mu|^2 / 3 when f(0) = 0, and
 * f0_fit_s = 2 dE_s B_s.
 *   q_fit   fit range in a.u. (> 0; the paper uses about 0.05-0.25 keV)
 *   coef    [n_states][3] = (A, B, C), host, required
 *   f0_fit  [n_states] host, or NULL (needs dE)
 */
int scff_dipole_fit(scff_ctx* ctx, double q_fit, const double* dE, double* coef, double* f0_fit);

/* ---- serving: continuous batching of independent requests -------------- */
typedef struct scff_server scff_server;

typedef struct {
    /* molecule (as scff_load_molecule) */
    int n_atoms;
    const double* xyz_bohr;
    int n_shells;
    const int* shell_atom;
    const int* shell_l;
    const int* shell_nprim;
    const double* exps;
    const double* coefs;
    int normalise;
    /* transitions (as scff_load_transitions) */
    int n_states;
    const double* T;
    /* evaluation */
    scff_grid grid;
    int precision;
    double screen_eps;
    double spin_factor;
    /* host outputs, owned by the caller, written when the request completes;
     * must stay valid until scff_server_wait reports completion */
    float* f;    /* [n_states][nx][ny][nz][2] or NULL */
    float* f2;   /* [n_states][nx][ny][nz] or NULL     */
} scff_request;

typedef struct {
    long long submitted, completed, failed, cancelled;
    long long queued, inflight;
    size_t admitted_bytes, budget_bytes, peak_admitted_bytes;
    long long peak_inflight;
    /* requests whose molecule was already loaded on the idle context that
     * served them (its load was skipped) */
    long long mol_cache_hits;
    /* time spent in each stage, summed over completed requests (ns):
     * [0] waiting for a prep thread, [1] prep (molecule, T, precompute),
     * [2] waiting for admission and a run slot, [3] run (tables, grid
     * kernel, copy into pinned staging), [4] copy to the caller's buffers */
    long long ns_stage[5];
    /* batch launches, the requests they carried, and graph executables
     * instantiated / reused with updated parameters */
    long long batches, batched_requests, graphs_instantiated, graphs_updated;
    /* batches run with eager launches because their graph capture failed */
    long long eager_batches;
} scff_server_stats;

/* Create a server on `device`.  A request is prepared (basis, pair
 * precompute, screening, packing: its exact device footprint is then known)
 * by one of 8 prep threads, admitted in FIFO order while the device bytes of
 * all admitted requests fit `hbm_budget_bytes` (0 = 64 GiB) and at most
 * `max_inflight` requests are admitted (1..64), and run by one of two batch
 * runners: the admitted requests waiting for a runner (up to half of
 * max_inflight, rounded up) join its next batch, so two batches overlap on
 * the device.  A batch's launches (each request's 1D tables, one persistent
 * grid kernel per kernel variant consuming the (request, tile) items of all
 * its requests from a device queue, split reductions, result copies) are
 * captured into a
 * HIP graph; an executable graph is kept per launch topology (up to 32 per
 * runner) and replayed with the next batch's parameters.  A request's
 * results are identical alone and in any batch.  A request larger than the
 * whole budget fails with SCFF_ENOMEM.
 * Device memory: the budget caps the admitted requests together with the
 * prepared requests waiting for admission (a new prep starts only while
 * both leave room, or when nothing is prepared ahead); on top of it come
 * the preps in progress (at most 8 requests) and the idle contexts kept for
 * reuse: up to (8 + max_inflight) of them, each holding at most
 * budget / (2 x that count) device bytes, so at most budget / 2 in total.
 * An idle context keeps the molecule of its last request in device memory:
 * a request on the same molecule (equal geometry, shells, exponents,
 * coefficients and normalise flag) is given that context and skips the
 * molecule load (host basis build and upload).
 * Results are copied from the device into pinned host staging buffers of
 * the server (kept for reuse until scff_server_destroy) and from there, by
 * copy threads, into the request's f / f2; a request completes when its
 * results are in the caller's buffers.  At most 2 x max_inflight requests
 * are running or waiting for that host copy at once.
 * device = -1 selects a scheduler test mode that touches
 * no GPU: requests are validated, admitted and completed exactly as above,
 * but nothing is computed and their outputs are left untouched. */
int scff_server_create(int device, size_t hbm_budget_bytes, int max_inflight,
                       scff_server** out);

/* Copy the request's inputs and enqueue it; returns a ticket (> 0). */
int scff_server_submit(scff_server* srv, const scff_request* req, unsigned long long* ticket);

/* Wait up to timeout_ns (< 0: forever) for a ticket.  Returns SCFF_OK when
 * the request finished (its status in *status: SCFF_OK or the error code),
 * SCFF_EBUSY on timeout.  latency_ns (may be NULL) receives submit-to-done
 * time.  A ticket can be waited for successfully once. */
int scff_server_wait(scff_server* srv, unsigned long long ticket, long long timeout_ns,
                     int* status, long long* latency_ns);

/* Cancel a queued (not yet admitted) request. SCFF_EBUSY if already running. */
int scff_server_cancel(scff_server* srv, unsigned long long ticket);

/* Counters of the server since its creation, copied into *out (caller-owned).
 * queued / inflight / admitted_bytes are the current values; the peaks,
 * totals and summed stage times cover its whole life.  SCFF_EINVAL on a
 * NULL argument.  Thread-safe. */
int scff_server_stats_get(scff_server* srv, scff_server_stats* out);

/* Message of the most recently failed request ("ticket N: ..."; "" if
 * none), copied into buf (at most len - 1 characters and a terminating NUL).
 * SCFF_EINVAL on a NULL argument or len == 0.  Thread-safe. */
int scff_server_last_failure(scff_server* srv, char* buf, size_t len);

/* Destroy the server: requests not yet running are cancelled, running ones
 * (and their host copies) finish first; then every context, stream and
 * staging buffer is released.  srv is invalid afterwards. */
void scff_server_destroy(scff_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* SCARFF_H */
