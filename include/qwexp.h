/*
 * qwexp -- exp(-i t H) psi on the n-qubit hypercube for MI355X (gfx950).
 *
 * H = H_P + gamma * H_G with H_P diagonal (Ising energies E(z)) and
 * H_G = sum_j X_j (section I of Hopkins & Kendon, "Numerical methods for the
 * simulation of quantum walks and quantum annealing").  The action is evaluated
 * as a Chebyshev series of exp(-i a x) (Bessel coefficients, Eq. cheb, or the
 * Caratheodory-Fejer correction of section II.C) by the matrix Clenshaw
 * recurrence (Alg. 2, Eq. recursion) with a matrix-free H_G (section II.D).
 *
 * Conventions shared by every entry point
 *   - Qubit j is bit j of the basis index z; s_j(z) = 1 - 2*bit_j(z).
 *   - Complex vectors are interleaved (re, im): complex64 = 2 x float,
 *     complex128 = 2 x double, i.e. torch.complex64 / torch.complex128 storage.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.  The caller owns all memory.
 *     The library allocates nothing on the device: all scratch comes from the
 *     caller's workspace (size from qw_workspace_bytes / the batched and
 *     gradient size queries).
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *     enqueue their kernels on it.  Host synchronisation of an action call:
 *       * the spectral bound (plain calls, qw_spectral_bound_*) is read back
 *         once, 16 bytes; this one wait also covers the upload of (h, J);
 *       * calls given (c, r) with the diagonal from (h, J) wait once for that
 *         upload unless the norm monitor's read-back follows;
 *       * the one-workgroup path (n <= 13, complex64 or complex128, no norm
 *         monitor) waits once more, at its end, for its coefficient upload;
 *       * the norm monitor reads back its K + 2 norms at the end (one wait);
 *       * timing != 0 waits for the call's last event.
 *     So a plain call of n >= 14 synchronises exactly once, at the read-back,
 *     before its Clenshaw passes are enqueued; they run asynchronously.
 *   - Errors: every call returns a qw_status; nothing is thrown across the ABI.
 *     qw_last_error() returns a thread-local message for the last failure.
 *   - Calls on distinct workspaces may run concurrently from different threads.
 */
#ifndef QWEXP_H
#define QWEXP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QW_OK = 0,
    QW_EINVAL = -1,    /* bad size, tolerance, pointer or non-finite scalar      */
    QW_ENOMEM = -2,    /* workspace smaller than required                        */
    QW_EHIP = -3,      /* a HIP runtime call failed                              */
    QW_EDIVERGE = -4,  /* the recurrence grew past its bound (radius too small)  */
    QW_ENOCONV = -5    /* coefficient setup did not converge                     */
} qw_status;

typedef enum { QW_CHEB = 0, QW_CF = 1 } qw_method;

/* Filled on the host before an action call returns (may be NULL).  The input
 * fields are `timing` and `monitor`; every other field is output. */
typedef struct {
    int n;              /* qubits                                                 */
    int K;              /* polynomial degree; K+1 coefficients                    */
    int passes;         /* global passes per Clenshaw term                        */
    int method;         /* qw_method actually used                                */
    double shift_c;     /* spectral shift c = (max E + min E)/2                   */
    double radius_r;    /* bound r on the spectral radius of H - cI               */
    double a;           /* t * r, the argument of the Bessel coefficients         */
    double trunc_bound; /* truncation bound (Chebyshev tail sum or CF estimate)   */
    double eval_bound;  /* a-priori evaluation-error bound, section II.B.3        */
    int timing;         /* in: 1 records HIP events on the stream around the setup
                           and the Clenshaw loop and synchronises at the end;
                           2 also records one after every pass (multi-pass path) */
    float setup_ms;     /* out (timing): bound, diagonal, coefficients            */
    float loop_ms;      /* out (timing): all Clenshaw terms and the final step    */
    float pass_ms[4];   /* out (timing 2): pass p summed over all terms           */
    int monitor;        /* in: nonzero measures ||b_k|| of every term (fused in the
                           last pass), fills eval_bound and checks the growth      */
    double growth;      /* out (monitor): max over k of ||b_k|| / its limit for a
                           valid bound (> 1 means QW_EDIVERGE)                     */
    double out_norm;    /* out (monitor): ||psi_out||                             */
    int otf_mask;       /* out: bit o set if the passes of orientation o rebuild
                           the diagonal from (h, J) instead of reading it         */
} qw_info;

/* ------------------------------------------------------------------------
 * Caller-supplied polynomials p(H~) psi, H~ = (H - c I) / r
 * ------------------------------------------------------------------------ */
typedef enum {
    QW_BASIS_CHEB = 0, /* p(x) = sum_k coef_k T_k(x), Clenshaw's recurrence (Alg. 2)  */
    QW_BASIS_MONO = 1  /* p(x) = sum_k coef_k x^k, Horner's rule (Alg. 1)             */
} qw_basis;

#define QW_POLY_KMAX 131072

/* psi_out = p(H~) psi_in for H = diag(E) + gamma sum_j X_j (section II.B, Alg. 1
 * and Alg. 2 with a caller-supplied polynomial; the Chebyshev case is the
 * evaluation of Eq. recursion with arbitrary coefficients).
 *   coef : host, 2 (K + 1) doubles, complex coefficients as (re, im) pairs,
 *          0 <= K <= QW_POLY_KMAX;
 *   c, r : shift and scale of H~.  r > 0 uses them as given (no spectral bound
 *          is computed, no read-back); r <= 0 computes the bound of
 *          qw_spectral_bound_* (c ignored), so that H~ has its spectrum in
 *          [-1, 1]; info->shift_c and info->radius_r report the pair used.  If
 *          the computed r is 0 the result is p(0) psi_in.
 * Everything else as qw_expm_action_*: same layouts, workspace
 * (qw_workspace_bytes), stream semantics, aliasing of psi_out and psi_in, and
 * the same pass kernels (Horner's rule runs the fused pass schedule with unit
 * scale and no b_{k+2} term).  No global phase is applied; info->monitor must be
 * 0 (QW_EINVAL otherwise).  Complex64: gamma / r is rounded to float. */
qw_status qw_poly_action_c64(int n, const float *diag, const double *h, const double *J, double gamma,
                             double c, double r, const double *coef, int K, qw_basis basis,
                             const void *psi_in, void *psi_out, void *workspace, size_t ws_bytes,
                             void *stream, qw_info *info);
qw_status qw_poly_action_c128(int n, const double *diag, const double *h, const double *J, double gamma,
                              double c, double r, const double *coef, int K, qw_basis basis,
                              const void *psi_in, void *psi_out, void *workspace, size_t ws_bytes,
                              void *stream, qw_info *info);

/* ------------------------------------------------------------------------
 * Time-dependent anneal, fourth-order commutator-free Magnus steps (sec. III.B)
 * ------------------------------------------------------------------------ */
typedef struct {
    int timing;            /* in: nonzero times the call with HIP events and
                              synchronises                                       */
    int steps;             /* out: steps taken                                    */
    int exponentials;      /* out: exponentials applied (two per step)            */
    long long terms;       /* out: sum of the Chebyshev degrees over all
                              exponentials (the matrix-vector products)          */
    double err_bound;      /* out: sum over steps of the bound on the leading
                              local error, b(t) h^5                              */
    double h_min, h_max;   /* out: smallest and largest step                      */
    double comm_bound;     /* out: the bound used for ||[H_P, sum_j X_j]||        */
    float total_ms;        /* out (timing)                                        */
} qw_cfet_info;

/* psi_out = U(T, 0) psi_in for H(t) = A(t) H_P + B(t) sum_j X_j, H_P the Ising
 * diagonal of (h, J), by the fourth-order commutator-free Magnus method the
 * paper proposes for annealing (sec. III.B): each step of length h applies
 *   exp(-i h (a1 H(t1) + a2 H(t2))) first, then exp(-i h (a2 H(t1) + a1 H(t2))),
 * t_{1,2} = t + (1/2 -+ sqrt(3)/6) h, a_{1,2} = 1/4 +- sqrt(3)/6, each an
 * action call of the Chebyshev path on tables prepared once.
 *   A_coef, B_coef : host, A_deg + 1 / B_deg + 1 monomial coefficients in
 *                    s = t / T (degrees 0..16), e.g. A = s, B = 1 - s;
 *   steps > 0      : that many equal steps, tol the total truncation budget of
 *                    the Chebyshev series (tol h / (2T) per exponential);
 *   steps == 0     : adaptive steps h(t) = (tol / (2 T b(t)))^(1/4) from the
 *                    bound b(t) on the leading local error h^5 E5 (derived by
 *                    series expansion; it uses ||H_P - c||, n and the bound
 *                    sum_j 2(|h_j| + sum_k |J_jk|) on ||[H_P, sum_j X_j]||), so no
 *                    trial steps are run; half of tol goes to the series;
 *   step_sizes     : host, may be NULL; receives the first step_cap step sizes;
 *   workspace      : as qw_workspace_bytes(n, 64 or 128, n >= 31 in complex64);
 *   psi_out        : may alias psi_in; every exponential after the first runs
 *                    in place on psi_out.
 * Synchronises the stream once (the energy range).  QW_ENOCONV if more than
 * 2^20 steps would be needed. */
qw_status qw_anneal_cfet4_c64(int n, const double *h, const double *J, const double *A_coef, int A_deg,
                              const double *B_coef, int B_deg, double T, int steps, double tol,
                              const void *psi_in, void *psi_out, double *step_sizes, int step_cap,
                              void *workspace, size_t ws_bytes, void *stream, qw_cfet_info *info);
qw_status qw_anneal_cfet4_c128(int n, const double *h, const double *J, const double *A_coef, int A_deg,
                               const double *B_coef, int B_deg, double T, int steps, double tol,
                               const void *psi_in, void *psi_out, double *step_sizes, int step_cap,
                               void *workspace, size_t ws_bytes, void *stream, qw_cfet_info *info);

/* Host-only: the bound b(t) on ||E5|| used for the adaptive steps, for the
 * energy range [emin, emax] of H_P. */
qw_status qw_cfet4_step_bound(int n, const double *h, const double *J, const double *A_coef, int A_deg,
                              const double *B_coef, int B_deg, double T, double emin, double emax, double t,
                              double *bound);

/* Chebyshev coefficients of exp(-i a x) on [-1, 1] (section II.B.1, Eq. cheb,
 * with a -> -a; section II.C for QW_CF).  Host only.
 *   alpha : host, kmax+1 doubles; receives alpha_0..alpha_K with
 *           c_m = (-i)^m alpha_m (Chebyshev: alpha_0 = J_0(a), alpha_m = 2 J_m(a)).
 *   K_out : host int, the degree K (smallest whose truncation bound <= tol).
 *   err   : host double (may be NULL), the truncation bound of Eq. TruncError
 *           (Chebyshev) or |lambda_cos| + |lambda_sin| (CF).
 * Returns QW_EINVAL for tol <= 0 or non-finite a, QW_ENOMEM if K > kmax. */
qw_status qw_cheb_coeffs(double a, double tol, qw_method method, int kmax,
                         double *alpha, int *K_out, double *err);

/* Bessel values J_0(a) .. J_mmax(a) by Miller's backward recurrence (section
 * II.B.1) in double precision, normalised by J_0 + 2 sum J_2m = 1.  Host only;
 * J: host, mmax+1 doubles. */
qw_status qw_bessel_j(double a, int mmax, double *J);

/* Workspace bytes for one action call on n qubits at precision 64 (complex64
 * state, float diagonal) or 128 (complex128, double diagonal).  on_the_fly != 0
 * sizes the variant that never stores the diagonal (complex64 with diag == NULL
 * and n >= 31). */
size_t qw_workspace_bytes(int n, int precision, int on_the_fly);

/* Shift c and bound r of H - cI (section II.A): c = (max E + min E)/2,
 * r = (max E - min E)/2 + n |gamma| (the induced 1-norm).
 *   diag : device, N = 2^n energies (float for _f32, double for _f64), or NULL
 *          to compute E(z) = sum_{j<k} J_jk s_j s_k + sum_j h_j s_j on device
 *          from h (host, n doubles) and J (host, packed row-major upper
 *          triangle, n(n-1)/2 doubles).  A NaN or infinite energy gives
 *          QW_EINVAL.
 *   workspace : device, >= qw_workspace_bytes(n, 64|128, 0) bytes.
 * Synchronises the stream (16-byte read-back). */
qw_status qw_spectral_bound_f32(int n, const float *diag, const double *h, const double *J,
                                double gamma, double *c, double *r,
                                void *workspace, size_t ws_bytes, void *stream);
qw_status qw_spectral_bound_f64(int n, const double *diag, const double *h, const double *J,
                                double gamma, double *c, double *r,
                                void *workspace, size_t ws_bytes, void *stream);

/* psi_out = exp(-i t (diag(E) + gamma sum_j X_j)) psi_in  (section I, Eq.
 * SchroedSol), global phase exp(-i t c) of the spectral shift restored.
 *   n       : 1..32.
 *   diag    : device, N energies (float for _c64, double for _c128), or NULL to
 *             generate them from h, J (host arrays as in qw_spectral_bound_*).
 *             With diag == NULL the fused passes of the two end orientations
 *             rebuild the diagonal inside every Clenshaw term from per-tile
 *             tables and no pass reads a stored one: complex64 from 26 qubits
 *             (n >= 31: it is never stored, and the on-the-fly workspace has no
 *             room for it; 26-30: the workspace still has), complex128 from 26
 *             to 30 qubits.  Otherwise complex128 stores it in the workspace
 *             (n = 32: the workspace is 172 GB, with psi 240 GB in all).  A
 *             recomputed value is summed in double and rounded once.
 *   psi_in  : device, N complex values; psi_out: device, N complex values; they
 *             may be the same buffer.
 *   tol     : truncation tolerance (absolute, for a unit-norm psi).
 *   method  : QW_CHEB or QW_CF.
 *   workspace : device, >= qw_workspace_bytes(n, 64|128, on_the_fly) bytes,
 *             256-byte aligned.
 *   info    : host, optional.
 * Complex64 rounds gamma/r towards zero to float and redefines r = gamma/that,
 * so the hypercube term carries no rounding; the normalised diagonal is
 * formed in double and rounded once to float.  Enqueues ~K*passes kernels on
 * stream after one synchronising 16-byte read-back. */
qw_status qw_expm_action_c64(int n, const float *diag, const double *h, const double *J,
                             double gamma, double t, const void *psi_in, void *psi_out,
                             double tol, qw_method method,
                             void *workspace, size_t ws_bytes, void *stream, qw_info *info);
qw_status qw_expm_action_c128(int n, const double *diag, const double *h, const double *J,
                              double gamma, double t, const void *psi_in, void *psi_out,
                              double tol, qw_method method,
                              void *workspace, size_t ws_bytes, void *stream, qw_info *info);

/* Timing aid for choosing pass plans (not part of the action): one complex64
 * hypercube pass of the Clenshaw recurrence (section II.D) over caller device
 * buffers of 2^n complex64 amplitudes, with fixed coefficients, enqueued on
 * stream; the caller times it (e.g. with events on the same stream).
 *   mode        : 0 START (reads b1, psi, d), 1 ADD (b1, acc), 2 FUSED (b1, acc,
 *                 psi, d; writes dst and dst2);
 *   tb, nt      : tile of 2^tb amplitudes and nt threads: (12, 1024),
 *                 (13, 1024), (13, 512) or (14, 1024);
 *   on_the_fly  : START / FUSED rebuild the diagonal (d unused; (13, 512) and
 *                 (14, 1024) tiles with L + h = tb);
 *   L, g0, h    : the tile's L contiguous low bits and its h flipped bits
 *                 g0 .. g0 + h - 1 (L = g0 = 0: the contiguous orientation);
 *   xcd_order   : blocks take tiles in XCD-major order;
 *   workspace   : device, qw_workspace_bytes(n, 64, 1) bytes (tables of the
 *                 rebuilt diagonal, cleared here).
 * Outputs may alias inputs as in the action (dst = acc, dst2 = b1).  QW_EINVAL
 * for a shape or orientation the kernels do not have. */
qw_status qw_time_pass_c64(int n, int mode, int tb, int nt, int on_the_fly, int L, int g0, int h, int xcd_order,
                           const void *b1, const void *acc, void *dst, void *dst2, const void *psi,
                           const float *d, void *workspace, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * action as qw_expm_action_c64, same kernels and results, with no workspace
 * argument.  Its scratch is a fixed 22 MiB device array inside the library,
 * one per GPU, held until the process ends, enough for n <= 20 qubits; larger n
 * returns QW_EINVAL with a message.  The array's device address is looked up
 * once per device (the device current at the call).  Every call on one GPU
 * shares that GPU's array and nothing in it needs clearing between calls, but
 * calls that overlap on one GPU (on different streams or threads) race on it
 * and must be serialised by the caller.  The call allocates nothing on the
 * device; host synchronisation as qw_expm_action_c64. */
qw_status qw_expm_action_c64_noalloc(int n, const float *diag, const double *h, const double *J,
                                     double gamma, double t, const void *psi_in, void *psi_out,
                                     double tol, qw_method method, void *stream, qw_info *info);

/* ---- batched form (section III.A: many instances per launch) ----------- */

/* One instance of a batch.  Couplings h (n doubles) then J (n(n-1)/2 doubles,
 * packed row-major upper triangle) start at off_hJ in the host coupling pool;
 * the complex64 input and output states start at off_psi / off_out
 * (counted in amplitudes, even) in the device state pools. */
typedef struct {
    int n;              /* qubits, 1..22                                         */
    int reserved;
    double gamma, t, tol;
    int64_t off_hJ, off_psi, off_out;
} qw_batch_item;

/* Schedule of a batched call (what qw_batched_tune_c64 chooses). */
typedef struct {
    long long wave_bytes;       /* working-set cap of a wave of multi-pass instances
                                   (20 B per amplitude; 0: all in one wave)       */
    int onchip_nmax;            /* instances with n <= this (12 or 13; 0 = 13) run
                                   whole in one workgroup                          */
    int concurrent;             /* 1: that launch runs on a side stream of default
                                   priority, beside the multi-pass launches        */
    signed char tile_class[23]; /* per n (index n), multi-pass instances: 0 = 2^13-
                                   amplitude tiles, 1024 threads; 1 = 2^12, 1024
                                   threads (13 <= n <= 20); 2 = 2^13, 512 threads;
                                   -1 = default (1 for n = 13, else 0)             */
} qw_batch_sched;

typedef struct {
    int timing;         /* in: nonzero times setup and recurrence with HIP events */
    int count, small_count, large_count, max_K, launches, waves;
    long long amp_terms;   /* sum over instances of 2^n K                         */
    long long wave_bytes;  /* working-set cap per wave used (0: one wave)         */
    float setup_ms;        /* (timing) bound, diagonals, coefficients, uploads    */
    float loop_ms;         /* (timing) the recurrence launches (graph replay)     */
    int onchip_nmax, concurrent;   /* the schedule used                           */
    int graph_cached;      /* 1: the instantiated graph of an earlier call with the
                              same launch sequence and workspace was replayed     */
    float graph_ms;        /* host time to capture and instantiate the graph (0
                              when cached); not part of setup_ms or loop_ms       */
    int class_count[3];    /* multi-pass instances per tile class                 */
    signed char tile_class[23];   /* class used per n (-1: none / one workgroup)  */
} qw_batch_info;

/* Workspace bytes for qw_expm_action_batched_c64 (0 if the batch is invalid). */
size_t qw_batched_workspace_bytes_c64(const qw_batch_item *items, int count, const double *hJ_pool);

/* psi_out_i = exp(-i t_i (H_P,i + gamma_i sum_j X_j)) psi_in_i for every item,
 * complex64, each instance with its own spectral shift, bound and coefficients
 * (degree chosen for its own tol).  Instances with n <= 13 (or 12) run in one
 * persistent on-chip launch; larger ones in grouped two-pass launches (one per
 * tile class and step) captured into a HIP graph (eager launches when stream
 * is NULL), which later calls with the same launch sequence and workspace
 * replay without capturing again (four graphs are kept per process; a call
 * that evicts the oldest waits for its device to finish all work first).  The
 * schedule comes from the tune file tune_cache (may be NULL: the default).
 *   items : host array of count items; hJ_pool: host doubles;
 *   psi_pool / out_pool : device complex64 pools (16-byte aligned; output
 *   ranges must not overlap each other or any input range);
 *   workspace : device, >= qw_batched_workspace_bytes_c64 bytes, 256-aligned.
 * Synchronises the stream (bound read-back, and at the end). */
qw_status qw_expm_action_batched_c64(const qw_batch_item *items, int count, const double *hJ_pool,
                                     const void *psi_pool, void *out_pool, qw_method method,
                                     void *workspace, size_t ws_bytes, const char *tune_cache,
                                     void *stream, qw_batch_info *info);

/* Same with an explicit schedule (sched may be NULL: the default);
 * use_graph = 0 launches eagerly.  QW_EINVAL for a tile class that cannot hold
 * a size of the batch. */
qw_status qw_expm_action_batched_c64_sched(const qw_batch_item *items, int count, const double *hJ_pool,
                                           const void *psi_pool, void *out_pool, qw_method method,
                                           void *workspace, size_t ws_bytes, const qw_batch_sched *sched,
                                           int use_graph, void *stream, qw_batch_info *info);

/* Autotuner (section III.A's batching, with tile shapes chosen per size):
 * times the batch under candidate schedules -- the tile class of each size
 * bucket (13-16, 17-18, 19-20, 21-22 qubits) in turn, the one-workgroup limit,
 * the side-stream launch, wave sizes of 512 / 256 / 128 MB -- keeping a change
 * when it is faster (HIP events around the recurrence, graph built first);
 * writes the best to *best (may be NULL) and appends "<size signature>
 * wave=<bytes> onchip=<n> conc=<0|1> classes=<per n 1..22> ms=<time>" to the
 * text file tune_cache (may be NULL). */
qw_status qw_batched_tune_c64(const qw_batch_item *items, int count, const double *hJ_pool,
                              const void *psi_pool, void *out_pool, void *workspace, size_t ws_bytes,
                              const char *tune_cache, void *stream, qw_batch_sched *best);

/* ---- anneal energy and gradient ----------------------------------------- */

typedef struct {
    int timing;            /* in: nonzero times the whole call with HIP events     */
    int passes;            /* global passes per Clenshaw / adjoint term            */
    int sum_K;             /* total degree over the segments                       */
    long long amp_terms;   /* sum_s 2^n K_s of the forward sweep                   */
    float total_ms;
} qw_grad_info;

/* Workspace bytes for qw_anneal_energy_grad_c64 (0 for invalid arguments).  The
 * size is fixed from a host bound on every segment's degree. */
size_t qw_anneal_workspace_bytes_c64(int n, const double *h, const double *J, int S, const double *gamma,
                                     const double *t, int ckpt_every);

/* Piecewise-constant anneal psi_s = exp(-i t_s (H_P + gamma_s sum_j X_j)) psi_{s-1},
 * s = 1..S, evaluated with Chebyshev coefficients (complex64), its energy
 * E = <psi_S|H_P|psi_S> and the gradient of E with respect to every gamma_s,
 * t_s, h_j and J_jk by the adjoint of the Clenshaw recurrence (single-precision
 * adjoint, double-precision reductions).  The spectral shift c, the bounds r_s
 * and the degrees K_s are held fixed (stop-gradient); they are piecewise
 * constant in the parameters.
 *   h, J       : host couplings (SK layout as above); gamma, t: host, S values.
 *   psi0       : device complex64 initial state (2^n amplitudes).
 *   ckpt_every : window of the b_k recomputation; b_k pairs are checkpointed
 *                every ckpt_every terms during the forward sweep (0: one
 *                window per segment, no checkpoints); < 0: every b_k of every
 *                segment is kept (sum_s K_s vectors of workspace) and the
 *                backward sweep recomputes nothing.  The results are
 *                bit-identical for every ckpt_every.
 *   E, dgamma (S), dt (S), dh (n), dJ (n(n-1)/2): host outputs.
 *   psiT_out   : device complex64, receives psi_S (may be NULL).
 * 1 <= n <= 28.  Synchronises the stream once per segment. */
qw_status qw_anneal_energy_grad_c64(int n, const double *h, const double *J, int S, const double *gamma,
                                    const double *t, const void *psi0, double tol, int ckpt_every,
                                    double *E, double *dgamma, double *dt, double *dh, double *dJ,
                                    void *workspace, size_t ws_bytes, void *stream, void *psiT_out,
                                    qw_grad_info *info);

/* Same as qw_expm_action_c64 / _c128 with the spectral shift c and bound r given
 * by the caller (no bound read-back).  r must bound the spectral radius of
 * H - cI: the call always monitors ||b_k|| (as info->monitor does, fused into
 * the last pass of each term), fills info->eval_bound, and returns QW_EDIVERGE
 * when a Clenshaw vector or the result exceeds the limit that holds for any
 * valid bound (section II.B.3 and |U_j| <= j + 1).  Synchronises at the end. */
qw_status qw_expm_action_c64_bounded(int n, const float *diag, const double *h, const double *J, double gamma,
                                     double t, double c, double r, const void *psi_in, void *psi_out,
                                     double tol, qw_method method, void *workspace, size_t ws_bytes,
                                     void *stream, qw_info *info);
qw_status qw_expm_action_c128_bounded(int n, const double *diag, const double *h, const double *J,
                                      double gamma, double t, double c, double r, const void *psi_in,
                                      void *psi_out, double tol, qw_method method, void *workspace,
                                      size_t ws_bytes, void *stream, qw_info *info);

const char *qw_last_error(void);

/* Host-only self check of the tile index maps used by the Clenshaw passes for
 * n qubits at precision 64 or 128: every (tile, element) pair must address each
 * amplitude exactly once and every flipped partner must stay inside its tile.
 * Returns the number of passes per term, or a negative code on a violation.
 * Launches nothing. */
int qw_debug_check_plan(int n, int precision);

/* Host-only: the sequence of Clenshaw passes for degree K >= 1 over P
 * orientations, as quadruples (mode 0 START / 1 ADD / 2 FUSED, orientation,
 * term k, final flag) written to out (4*cap ints).  Returns the number of
 * passes; nothing is written when it exceeds cap.  Launches nothing. */
int qw_debug_schedule(int K, int P, int *out, int cap);

/* Library version string. */
const char *qw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QWEXP_H */
