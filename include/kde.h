/*
 * kde.h -- C ABI of the MI355X von Mises KDE library (libkdepic.so).
 *
 * The library computes the data-parallel hot path of kernel-density-
 * estimation noise reduction for 1D periodic electrostatic particle-in-cell
 * (Wu & Qin, "Reducing Noise for PIC Simulations Using Kernel Density
 * Estimation Algorithm"):
 *
 *   - the least-squares cross-validation objective over a batch of candidate
 *     kernel concentrations (Sec. II.B, Eq. cv_def) and its argmin;
 *   - deposition of particles onto the grid with the von Mises kernel
 *     (Sec. II.A Eq. vonMises, Sec. II.B Eq. kde), with one global or a
 *     per-particle concentration (Sec. II.C, step 3);
 *   - interpolation of a grid field back to the particles with the same
 *     kernels (the field gather of the PIC step, Sec. III.A);
 *   - Silverman's particle-wise widths from a pilot density
 *     (Sec. II.C, Eq. adaptive_width and the geometric mean that follows).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Domain. Positions live on the periodic interval [0, L). The kernel of
 *   concentration kappa is the von Mises law written as a density in x:
 *       K_kappa(d) = exp(-2 kappa sin^2(pi d / L)) / (L * I0e(kappa)),
 *   I0e(k) = exp(-k) I0(k). Width h and concentration are related by
 *   kappa = (L / (2 pi h))^2. The grid has M nodes x_g = g L / M and every
 *   grid quantity is a point value at the nodes.
 * Shape. kde_domain.shape selects the kernel. KDE_SHAPE_VONMISES is the
 *   kernel above, parameterised by kappa. KDE_SHAPE_TRIANGLE is the
 *   first-order weighting of standard PIC with an adjustable width (Sec. I;
 *   Sec. IV compares it, with a CV-chosen width, against the other shapes):
 *       T_h(d) = max(0, 1 - |d|/h) / h,   0 < h <= L/2,
 *   |d| the periodic distance; h = L/M is standard PIC. Its two-fold
 *   convolution is the cubic B-spline scaled to h (plus its periodic image
 *   for h > L/4). For this shape every argument called kappa (kappa,
 *   kappa_i, kappas_h) carries half-widths h instead, each in (0, L/2].
 *   kde_adapt_widths, the batching form, sessions and the server are
 *   defined for the von Mises shape only.
 * Memory. Pointers named *_h are HOST pointers; every other pointer is a
 *   DEVICE pointer (HBM of the current HIP device). The caller owns all
 *   memory: inputs, outputs and the workspace. The library never allocates
 *   or frees device memory.
 * Precision. kde_domain.prec selects the element type of particle arrays
 *   (positions, per-particle concentrations, gathered values): KDE_F64 =
 *   double, KDE_F32 = float. Grid arrays and scalar results are always
 *   double. In the KDE_F32 form the per-pair and per-node kernel arithmetic
 *   runs in float, each term added to a per-thread double sum; Bessel
 *   normalisers, cross-block reductions and the final CV combination stay
 *   in double.
 * Streams. `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream). Every call only enqueues work on it and returns; results are
 *   valid once that work has completed. No call synchronises the device.
 * Positions. Positions outside [0, L) are wrapped on the device
 *   (x - L floor(x / L)); they are not rejected. Non-finite positions or
 *   per-particle concentrations propagate as NaN into the results and set
 *   a numeric status word (KDE_NUMERIC_* bits, kde_numeric_check).
 * Errors. Every entry point returns a kde_status. Arguments are checked on
 *   the host before anything is enqueued; on error nothing is enqueued and
 *   kde_last_error() returns a message (thread-local) naming the problem.
 *   The library never aborts and never throws across this interface.
 * Determinism. Reductions use fixed slots and a fixed order, with no
 *   floating-point atomics: the same inputs give bitwise identical results
 *   on every run.
 */
#ifndef KDE_H
#define KDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KDE_ABI_VERSION 6

typedef int32_t kde_status;

enum kde_status_code {
  KDE_OK = 0,
  KDE_E_INVALID_ARG = 1,   /* an argument breaks the rule stated for it        */
  KDE_E_WORKSPACE = 2,     /* workspace pointer NULL or smaller than required  */
  KDE_E_BUDGET = 3,        /* request larger than a serving budget            */
  KDE_E_AGAIN = 4,         /* result not ready yet                             */
  KDE_E_NOT_FOUND = 5,     /* unknown handle or ticket                         */
  KDE_E_HIP = 6,           /* a HIP runtime call failed; message has its text  */
  KDE_E_NUMERIC = 7,       /* non-finite value where a finite one is needed    */
  KDE_E_INTERNAL = 8,      /* broken internal invariant                        */
  KDE_E_CANCELLED = 9      /* request withdrawn before it ran                  */
};

enum kde_precision { KDE_F64 = 0, KDE_F32 = 1 };

/* Bits of a numeric status word: kernels that read positions or
 * per-particle concentrations record a non-finite position, and a
 * per-particle concentration that is non-finite or negative (for the
 * triangle: a half-width outside (0, L/2]). Such values do not fault and
 * are not rejected (they cannot be seen before the kernels run); the
 * results they touch become NaN and the word says so (kde_numeric_check,
 * kde_session_step, kde_server_poll, kde_batch_status). */
enum kde_numeric_flag { KDE_NUMERIC_POSITION = 1, KDE_NUMERIC_CONCENTRATION = 2 };

/* Operation codes for kde_workspace_size. */
enum kde_op {
  KDE_OP_CV_SCAN = 0,
  KDE_OP_DEPOSIT = 1,
  KDE_OP_GATHER = 2,
  KDE_OP_ADAPT = 3,
  KDE_OP_CV_FOURIER = 4,   /* kde_cv_scan_fourier    */
  KDE_OP_CV_REFINE = 5,    /* kde_cv_refine          */
  KDE_OP_ADAPT_EXACT = 6   /* kde_adapt_widths_exact */
};

/* Kernel shapes (see "Shape" above). */
enum kde_shape { KDE_SHAPE_VONMISES = 0, KDE_SHAPE_TRIANGLE = 1 };

/* The periodic domain [0, L), its M-node grid, the particle precision and
 * the kernel shape. Rules: L finite and > 0; 2 <= M <= 4096; prec a
 * kde_precision value; shape a kde_shape value; reserved 0. */
typedef struct kde_domain {
  double L;
  int32_t M;
  int32_t prec;
  int32_t shape;
  int32_t reserved;
} kde_domain;

/* Largest concentration a CV scan accepts (kde_cv_scan, the batching form,
 * sessions and requests): far beyond any resolvable width (kappa = 1e12 is
 * a width of L / (2 pi 10^6)), and it keeps every exponent of the pair sums
 * within the range the pair kernel's exponential handles without a clamp. */
#define KDE_MAX_CV_KAPPA 1e12

/* Largest number of candidate concentrations one kde_cv_scan accepts. */
#define KDE_MAX_KAPPAS 64

/* Version of this interface (KDE_ABI_VERSION of the built library). */
int32_t kde_abi_version(void);

/* Text of a status code (static storage). */
const char* kde_status_str(kde_status s);

/* Message of the last failed call on this thread ("" if none). */
const char* kde_last_error(void);

/*
 * kde_numeric_check -- the numeric status of the plain calls
 * (kde_cv_scan, kde_cv_scan_noalloc, kde_cv_scan_fourier, kde_cv_refine,
 * kde_deposit, kde_gather, kde_adapt_widths, kde_adapt_widths_exact). Their
 * kernels set KDE_NUMERIC_* bits in a status word the library keeps per
 * device. This call waits for `stream` (hipStream_t or NULL), takes the
 * word (reads and clears it with one atomic exchange, enqueued on `stream`)
 * and writes it to *flags_h: KDE_E_NUMERIC if any bit was set since the
 * previous check on this device, KDE_OK if none. The word is shared by every
 * stream and thread on the device, so a plain call on another stream may
 * set it too; sessions, batches and server requests keep words of their own.
 */
kde_status kde_numeric_check(void* stream, uint32_t* flags_h);

/*
 * kde_workspace_size -- bytes of device workspace an operation needs.
 *   op     : a kde_op value.
 *   dom    : domain (host pointer); M and prec matter for every op.
 *   N      : number of particles (>= 1; >= 2 for the CV ops).
 *   B      : number of concentrations for the CV ops (1..KDE_MAX_KAPPAS),
 *            ignored otherwise.
 *   bytes_h: receives the size; the workspace must be 256-byte aligned.
 * The size depends only on (op, M, prec, N, B). A workspace may be reused by
 * later calls once the work enqueued with it has completed (or on the same
 * stream, right away).
 */
kde_status kde_workspace_size(int32_t op, const kde_domain* dom, int64_t N, int32_t B,
                              size_t* bytes_h);

/*
 * kde_cv_scan -- least-squares cross-validation over candidate
 * concentrations (Sec. II.B, Eq. cv_def, with the two-fold convolution Kbar
 * of the kernel; the leave-one-out estimator of Eq. Ehat in the second term).
 *
 * For each b in [0, B):
 *   S1[b] = sum_{i<j} Kbar_{kappa_b}(x_i - x_j),
 *   S2[b] = sum_{i<j} K_{kappa_b}(x_i - x_j),
 *   cv[b] = (N Kbar_b(0) + 2 S1[b]) / N^2 - 4 S2[b] / (N (N - 1)),
 * where for the von Mises kernel
 *   Kbar_kappa(d) = I0(2 kappa |cos(pi d / L)|) / (L I0(kappa)^2)
 * and for the triangle of half-width h
 *   Kbar_h(d) = (B(d/h) + B((L - d)/h)) / h,  Kbar_h(0) = 2 / (3 h),
 * B the centred cubic B-spline.
 * argmin receives the smallest b with cv[b] == min cv (first minimum).
 *
 *   dom      : domain (host). M is not used by this op.
 *   N        : particles (>= 2).
 *   x        : device array of N positions, element type by dom->prec.
 *   B        : number of candidates, 1..KDE_MAX_KAPPAS.
 *   kappas_h : host array of B concentrations in [0, KDE_MAX_CV_KAPPA],
 *              strictly ascending (triangle: B half-widths in (0, L/2],
 *              strictly ascending).
 *   cv       : device, B doubles (output).
 *   sums     : device, 2B doubles [S1[0..B), S2[0..B)] (output) or NULL.
 *   argmin   : device, 1 int32 (output) or NULL.
 *   ws, ws_bytes: device workspace of at least
 *              kde_workspace_size(KDE_OP_CV_SCAN, dom, N, B) bytes.
 *   stream   : hipStream_t or NULL.
 * Terms whose exponent lies below -70 (each smaller than e^-70 times the
 * largest term of its sum) may be left out: the kernel skips them where
 * that saves work and keeps them where it does not (the sums differ from
 * the full ones by at most that bound per term). For the triangle, pairs
 * outside the support of a width (d >= 2 h) contribute exactly 0 and are
 * skipped.
 */
kde_status kde_cv_scan(const kde_domain* dom, int64_t N, const void* x, int32_t B,
                       const double* kappas_h, double* cv, double* sums, int32_t* argmin,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * kde_cv_scan_noalloc -- kde_cv_scan without a caller-given workspace, for
 * callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation. Same
 * arguments, rules, outputs and kernels as kde_cv_scan (the same bits);
 * the workspace is an array of KDE_CV_NOALLOC_MAX_BYTES the library holds
 * in device memory, one per device, from the library's load on that device
 * until the process ends. The call allocates nothing.
 *   Limit: a scan whose kde_workspace_size(KDE_OP_CV_SCAN, dom, N, B)
 *   exceeds KDE_CV_NOALLOC_MAX_BYTES is refused with KDE_E_WORKSPACE before
 *   anything is enqueued (24 MiB holds N up to 220,191 in double and
 *   1,015,616 in float at B = 32, up to 54,528 in either at B = 64).
 *   Concurrency: every call on one device uses that device's one array, so
 *   calls that overlap on a device (other streams or threads) race and give
 *   undefined results; calls enqueued on one stream are safe.
 */
#define KDE_CV_NOALLOC_MAX_BYTES (24u << 20)
kde_status kde_cv_scan_noalloc(const kde_domain* dom, int64_t N, const void* x, int32_t B, const double* kappas_h,
                               double* cv, double* sums, int32_t* argmin, void* stream);

/*
 * kde_deposit -- kernel density estimate at the grid nodes (Sec. II.B
 * Eq. kde; with per-particle concentrations the adaptive estimate of
 * Sec. II.C, step 3, each kernel normalised on its own):
 *   rho[g] = (1/N) sum_i K_{kappa_i}(x_g - x_i),  g = 0..M-1.
 *
 *   dom     : domain (host).
 *   N       : particles (>= 1).
 *   x       : device, N positions (dom->prec).
 *   kappa_i : device, N per-particle concentrations (dom->prec, each finite
 *             and >= 0), or NULL to use `kappa` for every particle.
 *             (Triangle: half-widths in (0, L/2]; a particle with a
 *             half-width outside that range makes the result NaN.)
 *   kappa   : global concentration (finite, >= 0), used when kappa_i is NULL
 *             (triangle: a half-width in (0, L/2]).
 *   rho     : device, M doubles (output).
 *   ws, ws_bytes: workspace of kde_workspace_size(KDE_OP_DEPOSIT, dom, N, 0).
 */
kde_status kde_deposit(const kde_domain* dom, int64_t N, const void* x, const void* kappa_i,
                       double kappa, double* rho, void* ws, size_t ws_bytes, void* stream);

/*
 * kde_gather -- a grid field at the particles with each particle's kernel:
 *   out[i] = (L/M) sum_g field[g] K_{kappa_i}(x_g - x_i).
 * It is the adjoint of kde_deposit: (L/M) sum_g F_g rho_g = mean_i out_i.
 *
 *   field : device, M doubles.
 *   out   : device, N values in dom->prec, in the order of x.
 *   other arguments as for kde_deposit; workspace from
 *   kde_workspace_size(KDE_OP_GATHER, dom, N, 0) (may be 0 bytes; ws may
 *   then be NULL).
 */
kde_status kde_gather(const kde_domain* dom, int64_t N, const void* x, const void* kappa_i,
                      double kappa, const double* field, void* out, void* ws, size_t ws_bytes,
                      void* stream);

/*
 * kde_adapt_widths -- Silverman's particle-wise widths from a pilot grid
 * density (Sec. II.C, Eq. adaptive_width and the geometric mean g), in
 * concentration form:
 *   f_i     = (1 - t) pilot[j] + t pilot[(j + 1) mod M],  j = floor(x_i/dx),
 *             t = x_i/dx - j (periodic linear interpolation of the pilot),
 *             floored at the smallest positive normal number of dom->prec;
 *   log g   = (1/N) sum_i log f_i;
 *   kappa_i = kappa_star * exp(2 alpha (log f_i - log g))
 * (the width factor (f_i/g)^(-alpha) on h becomes its inverse square on
 * kappa).
 *
 *   pilot      : device, M doubles (the pilot density on the grid).
 *   kappa_star : finite, > 0.      alpha : finite, >= 0 (0.5 in the paper).
 *   kappa_out  : device, N values in dom->prec (output).
 *   log_geomean: device, 1 double (output) or NULL.
 *   n_floored  : device, 1 int64 (output: particles whose pilot value was
 *                floored) or NULL.
 *   ws, ws_bytes: workspace of kde_workspace_size(KDE_OP_ADAPT, dom, N, 0).
 * dom->shape must be KDE_SHAPE_VONMISES.
 */
kde_status kde_adapt_widths(const kde_domain* dom, int64_t N, const void* x, const double* pilot,
                            double kappa_star, double alpha, void* kappa_out, double* log_geomean,
                            int64_t* n_floored, void* ws, size_t ws_bytes, void* stream);

/*
 * Fourier-moment route (von Mises shape only). On the circle the kernel is
 * the Fourier series K(d) = (1/L)(1 + 2 sum_{m>=1} rho_m cos(m 2 pi d / L)),
 * rho_m = I_m(kappa)/I_0(kappa), and its two-fold convolution has the
 * coefficients rho_m^2. With the sample's moments
 *   S_m = sum_j exp(i m theta_j),  P_m = |S_m|^2,  theta_j = 2 pi x_j / L,
 * the double sums of Eq. (cv_def) (Sec. II.B) become single sums over m:
 *   sum_{i,j} Kbar  = (N^2 + 2 sum_m rho_m^2 P_m) / L,
 *   sum_{i!=j} K    = (N^2 - N + 2 sum_m rho_m (P_m - N)) / L,
 *   cv(kappa)       = (2 A / N^2 - 4 C / (N (N - 1)) - 1) / L,
 * A = sum_m rho_m^2 P_m, C = sum_m rho_m (P_m - N): the same objective as
 * kde_cv_scan, in O(N M) work instead of O(N^2). M is where the series is
 * cut: the smallest m at which an upper bound on rho_m(kappa_max) (the
 * product of Amos's bounds on I_nu/I_{nu-1}) falls below 1e-18; rho_m
 * decreases in m and increases in kappa, so the same M serves every kappa.
 * The moments are FP64 sums in a fixed order, the rho_m come from the
 * backward recurrence of I_m/I_{m-1} in FP64 on the device; results are
 * deterministic. kappa must lie in [0, KDE_MAX_FOURIER_KAPPA] (M <= 9105).
 * The pair sums S1 = (N^2 - N + 2 sum_m rho_m^2 (P_m - N)) / (2 L) and
 * S2 = (N^2 - N + 2 C) / (2 L) are differences; where the diagonal
 * N Kbar(0) dominates them (few particles, narrow kernels) they carry an
 * absolute error of a few rounding units of N Kbar(0) (resp. N K(0)).
 */
#define KDE_MAX_FOURIER_KAPPA 1e6

/*
 * kde_cv_scan_fourier -- the CV objective of kde_cv_scan over B
 * concentrations through the Fourier moments (above). Arguments, outputs
 * (cv[B], sums[2B] or NULL, argmin or NULL: first minimum), errors and
 * synchrony as kde_cv_scan; dom->shape must be KDE_SHAPE_VONMISES, kappas
 * in [0, KDE_MAX_FOURIER_KAPPA] strictly ascending; dom->prec selects the
 * position type (the arithmetic is FP64 in both).
 *   ws, ws_bytes: kde_workspace_size(KDE_OP_CV_FOURIER, dom, N, B) bytes.
 */
kde_status kde_cv_scan_fourier(const kde_domain* dom, int64_t N, const void* x, int32_t B,
                               const double* kappas_h, double* cv, double* sums, int32_t* argmin,
                               void* ws, size_t ws_bytes, void* stream);

/*
 * kde_cv_refine -- the minimiser of the CV objective in concentration, not
 * limited to the list (Sec. II.B: the paper minimises the objective with a
 * Newton-type method). The list is scanned as by kde_cv_scan_fourier; with
 * b* its first minimum, Newton's method on u = log(kappa) solves
 * dCV/du = 0 between kappas[b*-1] and kappas[b*+1] (clipped to the list; a
 * kappa of 0 there is replaced by the smallest positive list value), with
 * bisection whenever a Newton step leaves the current bracket. dCV/dkappa
 * and d2CV/dkappa2 are series over the same moments, with
 *   d rho_m / d kappa = rho_{m+1} + (m / kappa) rho_m - rho_1 rho_m.
 * Where dCV/du has one sign over the bracket, the result is the end with
 * the lower objective. Every step runs on the device (no host round trip).
 *   result : device, 5 doubles (output): [kappa*, cv(kappa*), dCV/du at
 *            kappa*, Newton/bisection steps taken, b*].
 *   cv     : device, B doubles (output: the scan) or NULL.
 *   argmin : device, 1 int32 (output: b*) or NULL.
 * Other arguments, errors and synchrony as kde_cv_scan_fourier.
 *   ws, ws_bytes: kde_workspace_size(KDE_OP_CV_REFINE, dom, N, B) bytes.
 */
kde_status kde_cv_refine(const kde_domain* dom, int64_t N, const void* x, int32_t B,
                         const double* kappas_h, double* result, double* cv, int32_t* argmin,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * kde_adapt_widths_exact -- particle-wise concentrations as
 * kde_adapt_widths (Sec. II.C), with the pilot evaluated exactly at each
 * particle instead of interpolated from a grid:
 *   f_i = (1/N) sum_j K_{kappa_star}(x_i - x_j)   (all j, i included)
 *       = (1/L)(1 + (2/N) sum_m rho_m Re(conj(S_m) exp(i m theta_i))),
 * through the Fourier moments (above), O(N M) work. Then, as there,
 * f_i floored at the smallest positive normal number of dom->prec,
 * log g = (1/N) sum_i log f_i, kappa_i = kappa_star exp(2 alpha (log f_i -
 * log g)). The series form carries an absolute error of a few rounding
 * units of K(0) = (1/L)(1 + 2 sum_m rho_m) in f_i.
 *   kappa_star : in (0, KDE_MAX_FOURIER_KAPPA].   alpha : finite, >= 0.
 *   kappa_out  : device, N values in dom->prec (output).
 *   log_geomean: device, 1 double (output) or NULL.
 *   n_floored  : device, 1 int64 (output) or NULL.
 *   ws, ws_bytes: kde_workspace_size(KDE_OP_ADAPT_EXACT, dom, N, 0) bytes.
 * dom->shape must be KDE_SHAPE_VONMISES; dom->M is not used.
 */
kde_status kde_adapt_widths_exact(const kde_domain* dom, int64_t N, const void* x, double kappa_star,
                                  double alpha, void* kappa_out, double* log_geomean, int64_t* n_floored,
                                  void* ws, size_t ws_bytes, void* stream);

/*
 * Batching form. Many independent particle sets, each taken through the
 * whole path -- kde_cv_scan over one shared list of B concentrations (on the
 * set's first n_cv particles), kde_deposit at the set's kappa* (the pilot),
 * kde_adapt_widths with `alpha`, and kde_deposit with the resulting
 * per-particle concentrations -- in one hipGraph launch. The graph holds one
 * kernel per phase over the work units of every set, sets ordered by CV
 * cost (largest first): the pair and deposit phases launch one workgroup
 * per unit (a set's slot of tile pairs and concentration group, or a
 * particle chunk); the light phases (sort, reductions, finalize, widths)
 * launch about as many workgroups as the device keeps resident, which pull
 * units from per-phase device counters. Each set's outputs are bitwise
 * identical to those of the one-set calls on the same set.
 */
typedef struct kde_batch_set {
  int64_t N;          /* particles, >= 2                                        */
  const void* x;      /* device, N positions (element type: the batch's prec)   */
  double L;           /* period, finite and > 0                                 */
  int32_t M;          /* grid nodes, 2..4096                                    */
  int32_t reserved;   /* set to 0                                               */
  int64_t n_cv;       /* the CV scan uses the first n_cv particles (2..N); 0 = N */
  double* cv;         /* device, B doubles: the CV objective (output) or NULL   */
  double* pilot;      /* device, M doubles: pilot density at kappa* (output) or NULL */
  double* rho;        /* device, M doubles: adaptive density (output)           */
  void* kappa_i;      /* device, N values (prec): adaptive widths (output) or NULL */
  double* kappa_star; /* device, 1 double: the chosen concentration (output) or NULL */
} kde_batch_set;

typedef struct kde_batch kde_batch;

/* Plan a batch (host work only). The set array is copied; the device
 * buffers it points to must stay valid while the batch is run. Rules as
 * for the one-set calls: N >= 2, L finite > 0, 2 <= M <= 4096, x and rho
 * not NULL, 1 <= B <= KDE_MAX_KAPPAS ascending kappas in [0, KDE_MAX_CV_KAPPA], alpha
 * finite >= 0. *out_h receives the handle (NULL on error). */
kde_status kde_batch_plan(const kde_batch_set* sets_h, int32_t nsets, int32_t prec, int32_t B,
                          const double* kappas_h, double alpha, kde_batch** out_h);
/* Device workspace the batch needs (256-byte aligned). */
kde_status kde_batch_workspace_size(const kde_batch* b, size_t* bytes_h);
/* Enqueue the whole batch on `stream` as one graph launch. The first run
 * with a given workspace uploads the set descriptors into it (a blocking
 * copy) and captures the graph; later runs with the same workspace only
 * launch the graph. The workspace belongs to the batch between runs. */
kde_status kde_batch_run(kde_batch* b, void* ws, size_t ws_bytes, void* stream);
/* Numeric status of the last run: waits for `stream`, then writes each
 * set's KDE_NUMERIC_* bits to flags_h[k] (nsets words, the sets' order);
 * KDE_E_NUMERIC if any set met a non-finite position or concentration.
 * Every run clears the words first. */
kde_status kde_batch_status(kde_batch* b, uint32_t* flags_h, void* stream);
kde_status kde_batch_destroy(kde_batch* b);

/*
 * Resident PIC sessions (serving form). A session keeps one electron
 * population in HBM (inside a caller-owned arena) and advances it by the
 * KDE-PIC cycle of Sec. III.A with the width-update rule of Sec. II.D:
 * deposit with kappa_i -> net charge 1 - L rho -> three-point periodic
 * Poisson equation solved exactly (the mean charge removed) ->
 * centred field -> gather with kappa_i -> leapfrog push (electrons,
 * q/m = -1; v <- v - E dt, then x <- x + v dt, wrapped) -> Anderson-Darling
 * statistic of x/L against the uniform law, read by the host, whose
 * p-value drives the update rule (p > 2 thr: p_th = 2 thr; else p < p_th/2:
 * CV scan on the first n_cv particles gives h_target and p_th = p; then
 * always h_opt <- rate h_target + (1 - rate) h_opt) -> pilot deposit at
 * kappa* = (L / (2 pi h_opt))^2 -> adaptive widths for the next step.
 * Units follow the Birdsall convention (plasma frequency 1). Creation runs
 * the CV scan at t = 0 (h_opt = h_target at its optimum, p_th = 2 thr).
 * Every step waits once for the A^2 value (one 8-byte device-to-host copy)
 * and, when the rule fires, for the scan's argmin. The part of a step that
 * is the same every step (for KDE: deposit through the A^2 copy; for
 * standard PIC: the whole step) is captured into a HIP graph on the
 * session's stream at the first step and replayed by one graph launch per
 * step; its kernels are not seen by kde_timing.
 *
 * method KDE_PIC_STANDARD runs the same cycle as standard PIC, the
 * comparison method of Sec. III: linear ("cloud-in-cell") weighting for the
 * deposit and the gather (the triangle of half-width dx = L/M), no CV scan,
 * no test and no width update (B, n_cv, kappas_h, alpha, p_threshold and
 * adjust_rate are not used); its steps never wait on the host.
 *
 * Field energy (both methods): each step records W = (dx/2) sum_g E_g^2 of
 * the field it computes from the positions at the start of the step, so
 * entry n of the history is W(t_n), t_n = n dt, n = 0 .. history-1 (later
 * steps are not recorded). Sec. III.B reads the Landau damping rate off
 * log W (kde_damping_rate).
 */
typedef struct kde_pic_params {
  int64_t N;             /* particles, >= 2                                       */
  double L;              /* period, finite and > 0                                */
  int32_t M;             /* grid nodes, a power of two in [2, 2048]               */
  int32_t prec;          /* KDE_F64 or KDE_F32 (positions, velocities, widths)    */
  double dt;             /* time step, > 0                                        */
  int32_t B;             /* candidate concentrations of the CV scan, 1..64         */
  int32_t n_cv;          /* the scan uses the first n_cv particles, 2..N          */
  const double* kappas_h;/* host, B ascending concentrations in (0, KDE_MAX_CV_KAPPA] (copied) */
  double alpha;          /* Silverman sensitivity (0.5 in the paper)              */
  double p_threshold;    /* significance threshold of the test (0.01)             */
  double adjust_rate;    /* relaxation rate of the width (0.05)                   */
  int32_t method;        /* KDE_PIC_KDE (0) or KDE_PIC_STANDARD (1)               */
  int32_t history;       /* field-energy history length in steps, >= 0            */
} kde_pic_params;

enum kde_pic_method { KDE_PIC_KDE = 0, KDE_PIC_STANDARD = 1 };

typedef struct kde_session_info {
  int64_t step;          /* steps taken                                           */
  double p_th, h_opt, h_target;  /* update-rule state                             */
  double kappa_star;     /* concentration of the current pilot                    */
  double last_a2, last_p;/* last A^2 and its p-value                              */
  int64_t fired;         /* CV scans triggered by the rule after t = 0            */
  uint32_t numeric;      /* KDE_NUMERIC_* bits seen by the session's kernels      */
  uint32_t reserved;
} kde_session_info;

enum kde_session_field { KDE_SESSION_X = 0, KDE_SESSION_V = 1, KDE_SESSION_KAPPA = 2, KDE_SESSION_RHO = 3,
                         KDE_SESSION_E = 4, KDE_SESSION_ENERGY = 5 };

typedef struct kde_session kde_session;

/* Arena bytes a session with these parameters needs (256-byte aligned). */
kde_status kde_session_bytes(const kde_pic_params* p, size_t* bytes_h);
/* Create a session in `arena`: copies x0 and v0 (device, N values in
 * prec; positions in [0, L)), runs the t = 0 scan and widths, and returns
 * when that work is done. The copies are ordered after the work already
 * enqueued on `stream` (the caller's hipStream_t, or NULL), so x0 and v0
 * may come from kernels still running there; x0 and v0 may be released
 * once this call returns. The session owns one HIP stream (default
 * priority) for its own work. The arena must stay valid until
 * kde_session_destroy. KDE_E_NUMERIC (and no session) if x0 holds a
 * non-finite position. */
kde_status kde_session_create(const kde_pic_params* p, const void* x0, const void* v0, void* arena,
                              size_t arena_bytes, void* stream, kde_session** out_h);
/* Advance nsteps steps (returns when they are done). KDE_E_NUMERIC when a
 * step met a non-finite position or width (kde_session_info.numeric says
 * which); that step is counted, the rule and the widths are not updated.
 * KDE_E_INVALID_ARG while the session is attached to a server. */
kde_status kde_session_step(kde_session* s, int32_t nsteps);
kde_status kde_session_state(const kde_session* s, kde_session_info* info_h);
/* Copy a field to `dst` (device): X, V, KAPPA (N values in prec; KAPPA is
 * not kept by standard sessions), RHO, E (M doubles), ENERGY
 * (min(steps taken, history) doubles). */
kde_status kde_session_read(kde_session* s, int32_t what, void* dst);
/* Checkpoint to a host blob (blob_h NULL: *bytes_h receives the size) and
 * restore into a session of the same N, M, prec, method and history; a
 * restored session continues bitwise identically (energy history included). */
kde_status kde_session_save(kde_session* s, void* blob_h, size_t* bytes_h);
kde_status kde_session_restore(kde_session* s, const void* blob_h, size_t bytes);
kde_status kde_session_destroy(kde_session* s);

/*
 * kde_damping_rate -- the damping rate read off a field-energy history as in
 * Sec. III.B: the slope of log W through the first two peaks after t = 0,
 * a peak being an index n >= 1 with W[n-1] < W[n] >= W[n+1]:
 *   rate = (log W[p2] - log W[p1]) / ((p2 - p1) dt).
 * The energy decays at twice the rate of the field amplitude, so the rate
 * is 2 Im(omega) of the damped mode. Host arrays; runs on the host.
 *   energy_h : n >= 3 finite, positive values.    dt : > 0.
 *   rate_h   : receives the rate (NaN when W has fewer than two peaks).
 *   peaks_h  : receives [p1, p2] (-1 when missing) or NULL.
 */
kde_status kde_damping_rate(const double* energy_h, int64_t n, double dt, double* rate_h, int64_t* peaks_h);

/*
 * Request server (serving form): continuous batching of KDE solves beside
 * resident PIC sessions. A request is one particle set (a kde_batch_set:
 * positions, grid, outputs) taken through the whole path like one set of a
 * batch; the CV scan uses min(N, request n_cv, config n_cv) leading
 * particles (0 = no limit). Requests queue in arrival order; a scheduler
 * thread admits them into `nslots` slots (each a HIP stream of default
 * priority) whenever a slot is free and their workspaces fit in the free
 * part of the caller's arena (the HBM budget). A request's estimated work is
 * B n_cv (n_cv - 1) / 2 CV pair terms plus 2 N M deposit terms plus 5e7; it
 * is large from large_terms on. Large requests run alone, at most
 * large_slots at a time, in arrival order. Otherwise the oldest small
 * request heads a group, joined by up to max_batch - 1 later small ones
 * whose estimated work lies between a quarter and twice the head's; small
 * requests may pass waiting large ones. Slots run concurrently, one
 * workgroup per work unit, so they share the device with each other and
 * with the attached sessions' streams. Attached sessions (kde_server_attach)
 * are charged their arena bytes against the budget and stepped by the same
 * thread, one step in flight each, never blocking it. A request that alone
 * needs more than the whole budget is refused by kde_server_submit with
 * KDE_E_BUDGET. Results are bitwise the same whatever the mix. A failure
 * stays with its own work: a group whose device work fails completes its
 * requests with that status, a session whose step fails completes its
 * ticket, and the server goes on. Latency = completion noticed by the
 * scheduler minus submission, host steady clock. The request's device
 * buffers must stay valid until its ticket completes; the arena until
 * destroy.
 */
typedef struct kde_server_config {
  int32_t prec;          /* KDE_F64 or KDE_F32 for every request                  */
  int32_t B;             /* candidate concentrations, 1..64                       */
  const double* kappas_h;/* host, B ascending in [0, KDE_MAX_CV_KAPPA] (copied)   */
  double alpha;          /* Silverman sensitivity                                 */
  int64_t n_cv;          /* cap on the CV subsample (0 = none)                    */
  int32_t nslots;        /* concurrent slots, 1..64                               */
  int32_t max_batch;     /* requests per admission, 1..1024                       */
  int32_t large_slots;   /* large requests in flight at most (0 = 1)              */
  double large_terms;    /* estimated terms from which a request is large (0 = 2e9) */
} kde_server_config;

typedef struct kde_result {
  int32_t status;        /* KDE_OK, KDE_E_NUMERIC (a non-finite position or width
                            in the set), KDE_E_CANCELLED, KDE_E_HIP             */
  int32_t batch_size;    /* requests admitted together with this one              */
  double latency_s, queue_s, run_s;  /* total, waiting, on the device             */
  int64_t steps;         /* attached sessions: steps taken                        */
} kde_result;

typedef struct kde_server_stats_t {
  int64_t submitted, completed, rejected, launches;
  double mean_batch;     /* requests per admission                                */
  double p50_s, p99_s, mean_s, max_s;  /* latency of completed requests          */
  double wall_s;         /* first submission to last completion                   */
  double requests_per_s, pair_evals, particles;
  int64_t failed, cancelled;           /* requests that ended otherwise          */
  int64_t session_steps;               /* steps of attached sessions             */
  double session_p50_s, session_p99_s; /* their step latency (begin to done)     */
} kde_server_stats_t;

typedef struct kde_server kde_server;

kde_status kde_server_create(const kde_server_config* cfg, void* arena, size_t budget_bytes, kde_server** out_h);
/* Workspace bytes one request needs when admitted alone. */
kde_status kde_server_request_bytes(const kde_server* s, const kde_batch_set* req_h, size_t* bytes_h);
/* Queue a request. Its work follows everything already enqueued on `stream`
 * (the submitter's hipStream_t, or NULL) at the time of the call, so the
 * positions may come from kernels still running there. */
kde_status kde_server_submit(kde_server* s, const kde_batch_set* req_h, void* stream, uint64_t* ticket_h);
/*
 * kde_server_attach -- hand a resident session (Sec. III.A step with the
 * Sec. II.D rule) to the server for nsteps steps: the scheduler thread
 * advances it beside the requests, one step in flight at a time, charging
 * the session's arena bytes against the budget while it is attached
 * (KDE_E_BUDGET if they do not fit in the largest free block). The ticket
 * completes (kde_server_poll) when the steps are done, or with the status
 * of a step that failed (KDE_E_NUMERIC for non-finite values). Until then the
 * caller must not use the session. Step latencies enter kde_server_stats.
 */
kde_status kde_server_attach(kde_server* s, kde_session* session, int64_t nsteps, uint64_t* ticket_h);
/* Withdraw a queued request: KDE_OK (its result is KDE_E_CANCELLED),
 * KDE_E_AGAIN when it already runs (it will complete), KDE_E_NOT_FOUND
 * otherwise. For an attached session's ticket: KDE_OK, the session takes no
 * further step, and its ticket completes with KDE_E_CANCELLED (steps = those
 * taken) once the step in flight is done; the caller may then use the
 * session again. */
kde_status kde_server_cancel(kde_server* s, uint64_t ticket);
/* KDE_OK and the result once done, KDE_E_AGAIN while pending; a ticket that
 * ended otherwise returns its status (res_h filled). */
kde_status kde_server_poll(kde_server* s, uint64_t ticket, kde_result* res_h);
/* Block until the ticket completes, then as kde_server_poll. The server
 * must outlive every pending wait (destroy it only after they return). */
kde_status kde_server_wait(kde_server* s, uint64_t ticket, kde_result* res_h);
/* Wait until every submitted request has completed and every attached
 * session has taken its steps. */
kde_status kde_server_drain(kde_server* s);
kde_status kde_server_stats(kde_server* s, kde_server_stats_t* st_h);
/* Queued requests are dropped; running ones and the attached sessions'
 * steps in flight finish first. */
kde_status kde_server_destroy(kde_server* s);

/* Upper-tail p-value of an Anderson-Darling statistic under its limiting
 * law for a fully specified distribution (Anderson and Darling 1954),
 * computed on the host. */
kde_status kde_ad_pvalue(double a2, double* p_h);

/*
 * Tuning of the CV pair kernel, by particle count: chunk_h[k], the number
 * of concentrations evaluated per pass over a tile pair (4 or 8, or 16 in
 * double; KDE_E_INVALID_ARG otherwise), and
 * group_h[k], the number of concentrations one workgroup takes on (0 = all
 * of them; else a multiple of chunk_h[k] up to KDE_MAX_KAPPAS), so that a
 * tile pair is split over ceil(B / group) workgroups, which shortens the
 * critical path of small sets. group_h may be NULL (all zero). Entry k
 * applies to N <= n_max_h[k] (ascending); the last entry covers every
 * larger N. The choice changes speed only: each concentration accumulates
 * the same terms in the same order whatever the pass size or split, so
 * results are bitwise equal. The table is process-wide; set it before
 * launching work, not while calls on other threads are running.
 * kde_tune_get returns the entry used for N (group_h may be NULL). Until a
 * table is set, the library uses the one its autotuner measured on gfx950
 * (built in; the Python binding installs the same table from the package's
 * tune_gfx950.json).
 */
kde_status kde_tune_set(int32_t prec, int32_t count, const int64_t* n_max_h, const int32_t* chunk_h,
                        const int32_t* group_h);
kde_status kde_tune_get(int32_t prec, int64_t N, int32_t* chunk_h, int32_t* group_h);

#ifdef __cplusplus
}
#endif

#endif /* KDE_H */
