/*
 * cfet.h -- C ABI of the MI355X commutator-free exponential time-propagator
 * library (libcfet.so).
 *
 * The library propagates  i d/dt psi = H(t) psi  with
 *     H(t) = H0 + sum_k f_k(t) H_k                (paper Sec. 1, eq. DGL; A(t) = -i H(t))
 * by commutator-free exponential time-propagators (CFETs): one time step of
 * size dt is
 *     psi <- exp(Omega_1) exp(Omega_2) ... exp(Omega_s) psi        (Sec. 4, eq. Ucf)
 *     Omega_i = -i dt (a_i H0 + sum_k b_{i,k} H_k),
 *     a_i = sum_m g_{i,m},  b_{i,k} = sum_m g_{i,m} f_k(t + x_m dt)  (Sec. 7, eq. OmGLeg)
 * with the Gauss-Legendre points x_m of Table tab:GaussLeg and the weights
 * g_{i,m} built from the coefficient tables of Secs. 4-5.  exp(Omega_s) acts
 * on psi first.  Each exponential is computed by the Lanczos (Krylov)
 * technique of Sec. 8.1 with m basis vectors; all of it runs in HIP kernels
 * on one GPU.
 *
 * Conventions for every entry point
 *   - Return value: CFET_OK (0) or a positive CFET_E* code.  Nothing aborts
 *     and no C++ exception crosses this boundary.  cfet_last_error() gives a
 *     message for the last failure on a context (or, for ctx == NULL, the last
 *     failure of a context-less call on this thread).
 *   - Complex numbers are interleaved (re, im) float64 pairs, i.e. the layout
 *     of C99 double complex / torch.complex128.
 *   - Device pointers are HIP device allocations on the context's device.
 *     "Host or device" pointers are classified with hipPointerGetAttributes.
 *   - Work enqueued on a caller stream is stream-ordered: the call returns
 *     after enqueueing; faults found on the device (non-finite values,
 *     eigen-solver non-convergence) are latched and reported by the next call
 *     on the context or by cfet_stats().
 *   - A context is not thread-safe: calls on one context must not overlap.
 *     Its workspace (Krylov basis, internal vectors, barrier state) is shared
 *     by all its calls, so work it enqueues on different streams must not run
 *     concurrently either: use one stream per context, or order the streams.
 */
#ifndef CFET_H
#define CFET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFET_API __attribute__((visibility("default")))

#define CFET_VERSION 1
#define CFET_MAX_KRYLOV 64   /* largest Krylov dimension m */
#define CFET_MAX_TERMS 7     /* largest number of driven terms H_k */

enum {
  CFET_OK = 0,
  CFET_EINVAL = 1,        /* bad argument, shape or CSR structure */
  CFET_ENOMEM = 2,        /* device or host allocation failed */
  CFET_EDEVICE = 3,       /* HIP runtime error */
  CFET_ENONFINITE = 4,    /* NaN/Inf in input data or produced on the device */
  CFET_EUNSUPPORTED = 5,  /* valid request the library does not implement */
  CFET_ENOCONV = 6        /* small eigen-solver did not converge */
};

/* Coefficient tables (Tables 4thCFET, 6thCFET, 8thCoeff, 4thCFETOpt,
 * 6thCFETOpt; CF2:1 is the exponential midpoint rule, Sec. 4 eq. UCF2). */
typedef enum {
  CFET_CF2_1 = 0,
  CFET_CF4_2 = 1,
  CFET_CF4_3 = 2,
  CFET_CF4_3OPT = 3,
  CFET_CF6_4 = 4,
  CFET_CF6_5 = 5,
  CFET_CF6_5B = 6,
  CFET_CF6_6 = 7,
  CFET_CF6_5IMP = 8,
  CFET_CF6_5OPT = 9,
  CFET_CF6_6OPT = 10,
  CFET_CF8_11 = 11,
  CFET_NUM_SCHEMES = 12
} cfet_scheme;

/* Sparse Hermitian matrix in CSR.  row_ptr: int64[n+1] with row_ptr[0] = 0,
 * non-decreasing, row_ptr[n] = nnz.  col: int32[nnz] in [0, n).  val:
 * 2*nnz float64 (interleaved complex).  Columns need not be sorted; a
 * column may not repeat within a row.  Host or device pointers; read only
 * during cfet_create. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t *row_ptr;
  const int32_t *col;
  const double *val;
} cfet_csr;

/* Drive functions f_k(t), evaluated on the host in float64:
 *   COS       A cos(omega t + phi)
 *   SIN2_COS  A sin^2(pi t / Tp) cos(omega t + phi) for 0 <= t <= Tp, else 0
 *   PWC       u[j] for t_edges[j] <= t < t_edges[j+1], else 0 (npieces pieces,
 *             t_edges strictly increasing; host pointers, copied at create)
 *   SECH_COS  A cos(omega t + phi) / cosh((t - tc)/tau)  (pulse of Sec. 11.1,
 *             eq. BPulse)                                                    */
typedef enum {
  CFET_DRIVE_COS = 0,
  CFET_DRIVE_SIN2_COS = 1,
  CFET_DRIVE_PWC = 2,
  CFET_DRIVE_SECH_COS = 3
} cfet_drive_kind;

typedef struct {
  int32_t kind;
  double A, omega, phi, Tp, tc, tau;
  int32_t npieces;
  const double *t_edges; /* npieces + 1 entries (PWC only) */
  const double *u;       /* npieces entries (PWC only) */
} cfet_drive;

/* Flags for cfet_create. */
#define CFET_VALIDATE_HERMITIAN 0x1u /* check H = H^dagger for every matrix */
/* Execution path of cfet_propagate (default: chosen from the dimension).
 * All paths compute the same propagation; they differ in launch structure:
 * one kernel per Lanczos phase, one persistent single-workgroup launch per
 * call, or one persistent cooperative (grid-barrier) launch per call. */
#define CFET_FORCE_MULTIKERNEL 0x10u
#define CFET_FORCE_SINGLE 0x20u       /* if the rows fit one workgroup's registers */
#define CFET_FORCE_COOPERATIVE 0x40u  /* if the rows fit the co-resident blocks */
/* A forced persistent path that does not fit falls back to the multi-kernel
 * path; cfet_stats reports the path taken. */
/* Store the operator in sliced-ELL form (64-row slices, column-major, driven
 * terms first in each row) for the multi-kernel path.  Large dimensions
 * (n > 2^22, where only the multi-kernel path runs) default to
 * CFET_LAYOUT_SELL_SPLIT below, or CFET_LAYOUT_SELL_UNIFORM where the split
 * does not apply; this flag alone selects plain SELL-64. */
#define CFET_LAYOUT_SELL 0x100u
/* SELL-64 as above, plus per slice a shared part: an entry that at least 8
 * rows of a slice (all of them, in a slice of fewer rows) hold with the same
 * column offset (column = row XOR offset), term and value -- e.g. a site
 * operator's flip with one coupling -- is stored once per slice with a mask of
 * the rows holding it, instead of once per row.  Same results up to the order
 * of summation; detection runs on the host at cfet_create.  Implies
 * CFET_LAYOUT_SELL. */
#define CFET_LAYOUT_SELL_UNIFORM 0x200u
/* SELL-64 with shared parts, split into two passes per application, for
 * operators on n = 2^b rows (b >= 8) whose shared entries connect rows that
 * differ in a few bits (site operators of spin systems: column = row XOR
 * offset).  Shared entries whose offset has a bit at or above
 * min(16, b - 2) leave the first pass, so its gathers stay within 2^16 rows
 * of the row; a second pass visits the rows in a bit-permuted order in which
 * the rows such an entry connects lie in the same small block of the order,
 * and adds their contribution.  Each pass reads x once from memory instead of
 * re-reading far columns.  Same results up to the order of summation.  Kept
 * only when the second pass's entries are shared by at least 8 rows on
 * average (otherwise CFET_LAYOUT_SELL_UNIFORM); the default for n > 2^22.
 * Implies CFET_LAYOUT_SELL_UNIFORM. */
#define CFET_LAYOUT_SELL_SPLIT 0x800u
/* Above 4096 rows, and when the operator is stored as CSR only, cfet_create
 * may give the CSR paths a row order of their own (reverse Cuthill-McKee)
 * when that leaves at least a quarter fewer entries whose column lies in
 * another row block of the cooperative kernel; cfet_propagate, cfet_apply and
 * cfet_gradient then permute the caller's vectors in and out on the stream
 * (results equal up to the order of summation).  cfet_stats_t.reordered tells.
 * This flag keeps the caller's order. */
#define CFET_NO_REORDER 0x400u
/* Keep the merged CSR operator on the device also where the dimension
 * (n > 2^22) selects a SELL layout, so that cfet_gradient runs there (on the
 * multi-kernel CSR path; cfet_propagate keeps the SELL layout).  Costs 20
 * bytes per non-zero and 8 per row of device memory. */
#define CFET_KEEP_CSR 0x4000u

typedef struct cfet_ctx cfet_ctx;

/* Statistics of a context, accumulated over all cfet_propagate calls. */
typedef struct {
  int64_t n;                 /* Hilbert-space dimension */
  int64_t nnz_stored;        /* stored non-zeros of the merged operator */
  int64_t exponentials;      /* exponentials applied */
  int64_t matvecs;           /* H applications (sum of effective m) */
  int32_t min_m_eff;         /* smallest effective Krylov dimension seen */
  int32_t breakdowns;        /* exponentials that stopped early (beta ~ 0) */
  int32_t path;              /* last propagation path: 0 none, 1 multi-kernel,
                                2 single-workgroup, 3 cooperative */
  int32_t status;            /* latched device status (CFET_OK or code) */
  double last_norm;          /* ||psi|| after the last exponential */
  int64_t timed_launches;    /* launches timed with events (cfet_profile) */
  double timed_ms;           /* their summed event-measured duration */
  double segment_us[4];      /* persistent paths with the segment timers of cfet_profile: time of block 0 in
                                SpMV phases, reductions/barriers, small exponentials,
                                recombinations (microseconds, cumulative) */
  int32_t layout;            /* operator storage of the multi-kernel path: 0 merged CSR,
                                1 SELL-64, 2 SELL-64 with shared parts, 3 the same split
                                into two passes (CFET_LAYOUT_SELL_SPLIT) */
  int32_t reordered;         /* 1: the CSR paths run on their own row order (see
                                CFET_NO_REORDER) */
  int64_t matrix_bytes;      /* stored operator bytes one application of that layout
                                reads (values, columns, masks, row and slice data;
                                padding excluded) */
} cfet_stats_t;

/* Build a context for H(t) = H0 + sum_k f_k(t) Hk[k], k < nterms
 * (1 <= nterms <= CFET_MAX_TERMS).  All matrices must be n x n.  The matrices
 * are validated (shape, CSR structure, finiteness, optionally Hermiticity)
 * and copied into library-owned device memory on the current HIP device,
 * merged into one CSR whose entries carry their term index.  *out receives
 * the context (NULL on failure).  The caller owns the context and releases it
 * with cfet_destroy. */
CFET_API int cfet_create(const cfet_csr *H0, int32_t nterms, const cfet_csr *Hk,
                         const cfet_drive *fk, uint32_t flags, cfet_ctx **out);

/* Propagate psi in place over nsteps CFET steps of size dt starting at t0
 * (step n starts at t0 + n dt, computed fresh for each n).  psi_dev:
 * complex128[n] device buffer owned by the caller.  scheme: cfet_scheme.
 * krylov_m: Lanczos basis size, 1..CFET_MAX_KRYLOV (clipped to n).  dt may be
 * negative; nsteps == 0 is a no-op.  hip_stream: hipStream_t (NULL = default
 * stream).  Lanczos stops early at basis size j < m when
 * beta_j <= 1e-12 max_{k<=j}(|alpha_k| + beta_k); psi is never renormalised.
 * Enqueues only; returns CFET_EINVAL/ENOMEM/EDEVICE for host-visible
 * failures. */
CFET_API int cfet_propagate(cfet_ctx *c, void *psi_dev, double t0, double dt, int64_t nsteps,
                            int32_t scheme, int32_t krylov_m, void *hip_stream);

/* cfet_propagate for callers that cannot allocate device memory during the
 * call: code being captured into a HIP graph, tight serving loops, harnesses
 * that forbid allocation.  Same arguments, same result as cfet_propagate on
 * the multi-kernel path (CFET_FORCE_MULTIKERNEL), which it always takes; it
 * calls no hipMalloc/hipFree and allocates no host memory.  Its Krylov basis,
 * partial sums, Lanczos scalars and (for reordered operators) the state in the
 * stored row order live in a fixed 64 MiB device array of the library, one
 * per GPU, set up by the first cfet_create on that GPU and held until the
 * process ends: it needs
 *     (m - 1) n 16 bytes + (reordered: n 16) + about 100 KiB <= 64 MiB
 * (m = min(krylov_m, n)) and returns CFET_EINVAL with a message otherwise,
 * before enqueueing anything.  The array is shared by every call on a GPU
 * (and keeps the last call's contents): calls that overlap on one GPU --
 * concurrent streams, several threads, several contexts -- race and must be
 * serialised by the caller. */
CFET_API int cfet_propagate_static(cfet_ctx *c, void *psi_dev, double t0, double dt,
                                   int64_t nsteps, int32_t scheme, int32_t krylov_m,
                                   void *hip_stream);

/* cfet_propagate with every exponential taken by the Chebyshev technique
 * instead of Lanczos (Sec. 8.1; compared with Krylov in Sec. 8.2): with an
 * interval [lo, hi] holding the spectrum of H_i = a_i H0 + sum_k b_ik H_k --
 * the terms' Gershgorin intervals (computed at cfet_create) summed with the
 * weights, a negative weight swapping the ends -- sigma = (lo + hi)/2,
 * h = (hi - lo)/2, theta = dt h,
 *     psi <- e^{-i dt sigma} sum_{k=0..K} (2 - delta_k0) (-i)^k J_k(theta) T_k((H_i - sigma)/h) psi
 * with T_k by its three-term recurrence, K the smallest index whose tail
 * bound 2 (|theta|/2)^(K+1)/(K+1)! / (1 - |theta|/(2(K+2))) is at most tol
 * (so the error of each exponential is at most tol ||psi||).  Same step
 * driver, time grid and scheme as cfet_propagate; runs on the multi-kernel
 * path's operator layout (one apply and one update kernel per term), needs
 * three n-vectors of workspace (the context's Krylov workspace, grown to at
 * least that).  cfet_stats counts the exponentials, their K products
 * (matvecs) and the smallest K (min_m_eff); with cfet_profile on, the
 * applies are timed.  psi_dev: complex128[n] device buffer, in place; tol in
 * (0, 1); stream-ordered. */
CFET_API int cfet_propagate_chebyshev(cfet_ctx *c, void *psi_dev, double t0, double dt,
                                      int64_t nsteps, int32_t scheme, double tol,
                                      void *hip_stream);

/* Gradient of the final-state fidelity F = |<target|psi_N>|^2, psi_N the
 * state after nsteps CFET steps from psi0 (exactly the map of cfet_propagate:
 * same scheme, time grid and Lanczos exponentials with krylov_m vectors), with
 * respect to the amplitudes u[0..K-1] of the first driven term whose drive is
 * piecewise constant (CFET_DRIVE_PWC with K pieces).  u == NULL: the
 * amplitudes given at create; otherwise u (host, K finite values) replaces
 * them for this call only.
 * Method (adjoint of the discretised map): the weight of the term in
 * exponential i of step n is b = sum_m g_{i,m} f(t_n + x_m dt) (Sec. 7), so
 * db/du_p sums g_{i,m} over the Gauss points in piece p.  With the adjoint
 * state lambda (phi propagated back by the conjugate exponentials) and the
 * state psi before each exponential, its derivative is
 * <lambda| L(Omega, -i dt H_k) |psi>, L the Frechet derivative of the
 * exponential: the top-right block of exp([[Omega, D], [0, Omega]]), taken by
 * projecting that block-triangular operator on the Lanczos spaces of lambda
 * and psi (exact when the spaces are invariant).  The forward states are kept
 * every ceil(sqrt(nsteps)) steps and recomputed segment by segment.
 * psi0_dev, target_dev: complex128[n] device buffers (read only).  Writes
 * *F_out and dFdu_out[0..K-1] (host) and synchronises hip_stream.  Device
 * workspace O((sqrt(nsteps) s + 2 m) n), allocated for the call.  Needs the
 * CSR operator: kept for n <= 2^22, above that only with CFET_KEEP_CSR at
 * create (CFET_EUNSUPPORTED otherwise). */
CFET_API int cfet_gradient(cfet_ctx *c, const void *psi0_dev, const void *target_dev, double t0,
                           double dt, int64_t nsteps, int32_t scheme, int32_t krylov_m,
                           const double *u, int32_t K, double *F_out, double *dFdu_out,
                           void *hip_stream);

/* Result of cfet_select_dt. */
typedef struct {
  double dt;            /* selected step, T_total / nsteps */
  int64_t nsteps;       /* whole steps of size dt covering T_total */
  double c;             /* estimated error constant of eps = c T dt^N */
  double dt1, dt2;      /* probe steps window / n1, window / n2 */
  double diff;          /* largest ||x1 - x2|| over the checkpoints */
  double err_est;       /* c T_total dt^N (<= eps unless dt was capped at T_total) */
  double err_check;     /* error of dt over T_total from the verification runs
                           (NaN without verification) */
  double check_window;  /* their window: check_n1 steps of dt */
  int32_t order;        /* N of the scheme */
  int32_t n1, n2;       /* probe step counts over the window */
  int32_t check_n1, check_n2; /* step counts of the last verification runs (0: none) */
  int32_t rounds;       /* refinement rounds taken (see refine) */
} cfet_dt_choice;

/* Time step for an accuracy goal from two runs (Sec. 6.6; the error of an
 * order-N scheme over a time T behaves as eps = c T dt^N, Sec. 6.1).
 * Propagates copies of psi0 over the probe window [t0, t0 + window] with n1
 * steps and with n2 = J round((n1 / J) ratio^(1/N)) steps (at least n1 + J;
 * J = checkpoints, n1 a multiple of J), takes the largest distance d of the
 * two states at the J checkpoints t0 + j window / J, and sets
 *     c = d / (window |dt1^N - dt2^N|),   dt = (eps / (c T_total))^(1/N),
 * capped at T_total and rounded down to T_total / nsteps.  verify != 0 runs
 * the window stretched to whole multiples of J steps of the selected dt, with
 * dt and with the step of the same ratio below it, and reports their distance
 * d' scaled to the error of dt over T_total:
 *     err_check = d' dt^N / (dt^N - dt'^N) * T_total / check_window.
 * refine > 0 (needs verify): while err_check > eps, at most refine times, the
 * verification pair becomes the probe -- c = d' / (check_window |dt^N - dt'^N|),
 * a new (smaller) dt, a new verification; the output describes the last
 * round.  This catches probes taken where the error does not yet follow dt^N.
 * ratio = (dt1 / dt2)^N is meant to lie in 2 .. 3.  Every run is a
 * cfet_propagate with the given scheme and krylov_m on hip_stream.
 * psi0_dev: complex128[n] device buffer (read only).  Writes *out (host) and
 * synchronises hip_stream; device workspace of two state vectors, allocated
 * for the call.  CFET_EINVAL for window, T_total, eps <= 0, ratio <= 1,
 * checkpoints < 1, n1 not a positive multiple of checkpoints, refine < 0 or
 * refine > 0 without verify. */
CFET_API int cfet_select_dt(cfet_ctx *c, const void *psi0_dev, double t0, double window,
                            int32_t n1, int32_t checkpoints, double ratio, int32_t scheme,
                            int32_t krylov_m, double T_total, double eps, int32_t verify,
                            int32_t refine, cfet_dt_choice *out, void *hip_stream);

/* y = (a H0 + sum_k b[k] Hk[k]) x on the device (the weighted apply that the
 * Lanczos recursion uses; Sec. 8: the sparsity pattern of the sum is the
 * union of the patterns).  x_dev, y_dev: complex128[n] device buffers, must
 * not overlap.  b: host array of nterms doubles.  Stream-ordered. */
CFET_API int cfet_apply(cfet_ctx *c, const void *x_dev, void *y_dev, double a, const double *b,
                        void *hip_stream);

/* Synchronise the context's last stream and report statistics and the
 * latched device status (which this call clears). */
CFET_API int cfet_stats(cfet_ctx *c, cfet_stats_t *s);

/* Release all device and host memory of the context (synchronises). */
CFET_API int cfet_destroy(cfet_ctx *c);

CFET_API const char *cfet_last_error(const cfet_ctx *c);

/* Kernel timing for measurement: with enable != 0, cfet_propagate records a
 * HIP event pair on the caller's stream around every launch of its dominant
 * kernel -- the Lanczos SpMV on the multi-kernel path (both launches of a
 * split layout between one event pair; the apply of each term with
 * cfet_propagate_chebyshev), the whole persistent kernel on the
 * single-workgroup and cooperative paths, also its launches inside
 * cfet_gradient -- (up to max_launches
 * pairs; later launches run untimed), and cfet_stats reports the count and
 * summed duration.  enable == 2 records the events only; any other nonzero
 * value also runs the persistent kernels' segment timers (cfet_stats
 * segment_us), which read a clock in block 0 several times per Lanczos
 * iteration and so lengthen the kernel slightly.  The events add a little
 * launch overhead, so throughput is measured with timing off.  enable == 0
 * releases the events. */
CFET_API int cfet_profile(cfet_ctx *c, int32_t enable, int32_t max_launches);

/* Host-side view of the library's own scheme data: s (exponentials), M
 * (Gauss-Legendre points), the nodes x[M] and the weights g[s*M] (row-major,
 * g[i*M + m]).  Any output pointer may be NULL.  Sec. 7, eq. OmGLeg. */
CFET_API int cfet_scheme_info(int32_t scheme, int32_t *s, int32_t *M, double *x, double *g);

/* Per-step weights exactly as cfet_propagate uses them: a[i] (i < s) and
 * b[(n*s + i)*nterms + k] for steps n < nsteps.  Host arrays. */
CFET_API int cfet_step_weights(const cfet_ctx *c, double t0, double dt, int64_t nsteps,
                               int32_t scheme, double *a, double *b);

/* c = exp(-i dt T) e_1 for the real symmetric tridiagonal T with diagonal
 * alpha[k] and off-diagonal beta[k-1] (Sec. 8.1: the exponential of the small
 * projected matrix), computed by the device kernel that the propagator uses.
 * alpha_dev, beta_dev: float64 device arrays; c_dev: complex128[k] device
 * array; 1 <= k <= CFET_MAX_KRYLOV.  Stream-ordered; a convergence failure is
 * reported through *status_dev (int32 device scalar: 0 or CFET_ENOCONV). */
CFET_API int cfet_tridiag_expm(const double *alpha_dev, const double *beta_dev, int32_t k,
                               double dt, void *c_dev, int32_t *status_dev, void *hip_stream);

CFET_API int cfet_version(void);

/* ---------------------------------------------------------------------------
 * Batched propagation: many independent trajectories advanced together.
 *
 * Every instance t is its own problem  i d/dt psi_t = (H0_t + sum_k f_tk(t)
 * H_tk) psi_t  with its own drives and state; all share the scheme, the time
 * grid and the Krylov bound of a call.  Operators live in one table and
 * instances refer to them by index, so an operator used by many instances
 * (e.g. sum_i sigma^x_i of one chain length) is stored and streamed once for
 * all of them: instances with the same driven operators and dimension are
 * grouped (at most 64 per group) and their vectors interleaved, and each
 * Lanczos phase is one kernel over every instance of the batch.  The
 * exponentials are those of cfet_propagate (Sec. 8.1); with tol > 0 the
 * Krylov dimension is chosen per instance and per exponential: the recurrence
 * stops after j < m vectors when  |dt| beta_j |e_j^T exp(-i dt T_j) e_1| <= tol
 * (an a-posteriori estimate of the Krylov error relative to ||psi||; the
 * paper fixes m and leaves this choice open, Sec. 12), or by the breakdown
 * rule of cfet_propagate.  One CFET step is captured once as a HIP graph and
 * replayed.
 * ------------------------------------------------------------------------- */
typedef struct cfet_batch cfet_batch;

typedef struct {
  int32_t h0;                         /* operator index of H0 */
  int32_t nterms;                     /* driven terms, 0..CFET_MAX_TERMS */
  int32_t hk[CFET_MAX_TERMS];         /* operator indices of H_1..H_nterms */
  cfet_drive fk[CFET_MAX_TERMS];      /* their drives (PWC arrays: host, copied) */
} cfet_instance;

/* Flags for cfet_batch_create (CFET_VALIDATE_HERMITIAN applies as well). */
#define CFET_BATCH_NO_GRAPH 0x1000u     /* enqueue every kernel instead of graph replays */
#define CFET_BATCH_NO_AUTOTUNE 0x2000u  /* skip the launch-layout timing at create */

typedef struct {
  int32_t ninst;          /* instances */
  int32_t ngroups;        /* groups sharing operator reads */
  int64_t total_dim;      /* sum of the instance dimensions */
  int64_t matvecs;        /* H applications, summed over instances */
  int64_t exponentials;   /* exponentials, summed over instances */
  int64_t breakdowns;     /* exponentials stopped by the breakdown rule (or psi = 0) */
  int64_t early_stops;    /* exponentials stopped by the error estimate */
  int32_t min_m_eff;      /* smallest / largest Krylov dimension used */
  int32_t max_m_eff;
  int32_t status;         /* latched device status (cleared by this call) */
  int32_t unroll;         /* launch layout chosen at create: rows per lane and pass */
  int32_t graph;          /* 1 if the last call replayed the step graph */
  int32_t block_threads;  /* launch layout chosen at create: threads per block (128, 256, 512) */
  double tune_us[12];     /* create-time timing (us) of one product, its reduction and
                             the three-term update, [i * 4 + j] for 128, 256, 512
                             threads per block (i) and 2, 4, 8, 16 rows per lane and
                             pass (j); 0 if not timed.  The layout kept is, among those
                             within 3 % of the fastest, the one with the most rows per
                             block, then the fewest threads per block */
} cfet_batch_stats_t;

/* Build a batch.  ops: nops CSR matrices (host or device arrays, copied and
 * validated as by cfet_create).  inst: ninst instances.  The operators of
 * one instance must have the same dimension (< 2^29).  Times the launch
 * layouts once on the device unless CFET_BATCH_NO_AUTOTUNE.  *out receives
 * the batch (NULL on failure); release it with cfet_batch_destroy. */
CFET_API int cfet_batch_create(int32_t nops, const cfet_csr *ops, int32_t ninst,
                               const cfet_instance *inst, uint32_t flags, cfet_batch **out);

/* Propagate every instance over nsteps CFET steps of size dt from t0.
 * psi_dev: complex128 device buffer holding the instances' states one after
 * another in instance order (length = sum of their dimensions), updated in
 * place.  krylov_m: 1..CFET_MAX_KRYLOV (upper bound when tol > 0; clipped to
 * each instance's dimension).  tol >= 0 (0: fixed m).  Stream-ordered; device
 * faults are latched and reported by cfet_batch_stats. */
CFET_API int cfet_batch_propagate(cfet_batch *b, void *psi_dev, double t0, double dt,
                                  int64_t nsteps, int32_t scheme, int32_t krylov_m, double tol,
                                  void *hip_stream);

/* Fix the launch layout of the batch's row kernels instead of the one chosen
 * at create (tests, reproducible layouts): block_threads 128, 256 or 512,
 * rows_per_lane 2, 4, 8 or 16.  Results differ between layouts only in the
 * order of the block-partial sums.  Synchronises with the batch's last call;
 * the next call re-records its step graph.  CFET_EINVAL for other values. */
CFET_API int cfet_batch_set_layout(cfet_batch *b, int32_t block_threads, int32_t rows_per_lane);

/* Synchronise and report statistics; returns the latched device status. */
CFET_API int cfet_batch_stats(cfet_batch *b, cfet_batch_stats_t *s);

/* Synchronise and write each instance's cumulative H applications to out
 * (int64[ninst], instance order). */
CFET_API int cfet_batch_instance_matvecs(cfet_batch *b, int64_t *out);

CFET_API int cfet_batch_destroy(cfet_batch *b);

/* Message of the last failure on b (b == NULL: last batch call on this thread). */
CFET_API const char *cfet_batch_last_error(const cfet_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* CFET_H */
