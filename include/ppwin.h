/*
 * ppwin: frequency-window solver for the first- and second-order particle-hole
 * polarization propagator on one AMD Instinct MI355X (gfx950).
 *
 * The library computes, without assembling any response matrix, the product
 * sigma = M X of the particle-hole response matrix
 *
 *     M = [[A, B], [B, A]],  metric Sigma = diag(S, -S)
 *
 * (generalized eigenvalue equation of the Theory section, "Second-order
 * approximation of the polarization propagator") with a block of trial
 * vectors, and drives with it the frequency-dependent inverse-Krylov /
 * folded-spectrum solve of the subsection on interior eigenvalues: the roots of
 * M z = omega Sigma z nearest a chosen omega0, their eigenvectors and dipole
 * oscillator strengths.
 *
 * Scope: closed-shell singlet, real orbitals, density-fitted two-electron
 * integrals (pq|rs) = sum_P B_Ppq B_Prs (Results section), particle-hole
 * dimension N = n_occ * n_vir.  Orders: 0 (A = eps_a - eps_i, B = 0, S = 1),
 * 1 (singlet TDHF: A1 = 2(ia|jb) - (ij|ab), B1 = 2(ia|jb) - (ib|ja)), 2 (the
 * MP2-ground-state corrections S2, A2, B2 of the second-order equations, with the
 * W_N cross terms included in A as in B and the symmetrized double commutator;
 * MP2 amplitudes t_ij^ab = (ia|jb)/(eps_i + eps_j - eps_a - eps_b) are rebuilt
 * from B in occupied strips and never stored unless requested).
 *
 * Conventions shared by every entry point
 *  - particle-hole vectors are row-major [n_occ][n_vir] doubles (index i*v + a);
 *    a 2N vector is [X; Y] = two such blocks, X first.
 *  - unless PP_DEVICE_PTRS is given, pointers are host pointers; results are
 *    written to caller memory only, never retained.
 *  - every call returns a pp_status; no exception crosses the ABI.  On error the
 *    message is kept in the handle (pp_last_error) and outputs are unspecified
 *    unless the code says otherwise (PP_ENOTCONV writes all outputs).
 *  - a handle is used by one host thread at a time; the server object is
 *    thread-safe.
 */
#ifndef PPWIN_H
#define PPWIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PP_OK = 0,
  PP_EINVAL = 1,     /* bad argument (sizes, NaN/Inf in inputs, NULL pointer) */
  PP_ENOMEM = 2,     /* the request does not fit the HBM budget of the handle/server */
  PP_ENOTCONV = 3,   /* solve stopped at max_cycles; outputs written, info->converged flags 0 */
  PP_EUNSTABLE = 4,  /* A-B, A+B or S not positive definite in the subspace (complex roots) */
  PP_EDEVICE = 5,    /* HIP runtime error; message kept */
  PP_ENOTSUP = 6,    /* option combination not supported */
  PP_EPENDING = 7    /* server request not finished yet (pp_server_poll) */
} pp_status;

typedef enum {
  PP_FP64 = 0,       /* every contraction in FP64 on FP64 matrix cores */
  PP_FP32 = 1,       /* subspace products in FP32 matrix cores, FP64 residual refinement */
  PP_SPLIT_BF16 = 2  /* as PP_FP32, with the amplitude contraction as split-BF16 products: each
                        FP32 operand split into two BF16 parts, three BF16 MFMA products with FP32
                        accumulation (relative error about 2^-16); FP64 residual refinement */
} pp_precision;

/* How a window solve isolates the roots near omega0 (pp_options.method). */
typedef enum {
  PP_FOLDED = 0,     /* inverse Krylov basis from weighted-Jacobi steps of the shifted pencil,
                        folded-spectrum selection (the interior-eigenvalue subsection) */
  PP_RIESZ = 1       /* Riesz projector (the section on its connection to the method): the
                        block is filtered by trapezoidal quadrature of the contour integral of
                        (z Sigma - M)^-1 Sigma on a circle around omega0, each shifted system
                        solved by diagonal-preconditioned conjugate-orthogonal CG */
} pp_method;

/* pp_sigma flags */
#define PP_APPLY_METRIC 1u  /* return Sigma X instead of M X */
#define PP_DEVICE_PTRS 2u   /* X and out are device pointers */
#define PP_ASYNC 4u         /* return once the product is enqueued (with PP_DEVICE_PTRS only) */
#define PP_REDUCED 8u       /* contractions in the handle's reduced precision (opt->precision PP_FP32
                               or PP_SPLIT_BF16 at setup; PP_ENOTSUP on an FP64 handle); the
                               orbital-energy terms and the final combination stay FP64 */

typedef struct pp_handle pp_handle;

/* One closed-shell system.  All arrays are read during pp_setup only and copied
 * into device memory the handle owns; the caller may free them on return. */
typedef struct {
  int32_t n_occ, n_vir, n_aux;
  int32_t order;            /* highest order the handle serves: 0, 1 or 2 */
  const double* eps;        /* [n_occ + n_vir] orbital energies, occupied first (Ha) */
  const double* B_oo;       /* [n_aux][n_occ][n_occ] DF factors, symmetric in the last two */
  const double* B_ov;       /* [n_aux][n_occ][n_vir] */
  const double* B_vv;       /* [n_aux][n_vir][n_vir], symmetric in the last two */
  const double* dip;        /* [3][n_occ][n_vir] dipole integrals (NULL: no strengths) */
  int32_t device_ptrs;      /* nonzero: the arrays above are device pointers */
} pp_system;

typedef struct {
  int32_t precision;        /* pp_precision used by the subspace products (default FP64) */
  int32_t store_amplitudes; /* 1: keep all amplitude strips (o^2 v^2 doubles); 0: rebuild per
                               product; -1 (default): keep them when they fit the budget */
  int32_t strip_rows;       /* occupied rows per amplitude strip (0 = chosen from the budget) */
  double tol;               /* residual tolerance |(M - theta Sigma) y| / |y| (default 1e-9) */
  int32_t block;            /* block size (0: n_roots + 2; 2 n_roots for PP_RIESZ) */
  int32_t krylov_steps;     /* basis vectors per cycle: corrections + (krylov_steps-1)
                               weighted-Jacobi steps (default 2) */
  int32_t max_basis;        /* largest subspace (default 480, at most 512) */
  int32_t max_cycles;       /* default 200 */
  double d_clamp;           /* smallest |diagonal| of the Jacobi splitting (default 1e-4 Ha) */
  uint64_t hbm_budget;      /* bytes the handle may allocate (0: 90% of free device memory) */
  int32_t device;           /* HIP device ordinal */
  void* stream;             /* hipStream_t to run on (NULL: a stream owned by the handle) */
  uint64_t seed;            /* start-block perturbation seed */
  int32_t tda;              /* nonzero: Tamm-Dancoff problem, B = 0 (A z = omega S z), the
                               A-only variant of the error-analysis subsection (Discussion) */
  int32_t correlated_f;     /* nonzero: oscillator strengths from the property vector
                               F_k = <[q_k, mu]> over the MP2 ground state (Theory section,
                               the numerator of the propagator), which through second order is
                               the metric applied to mu: F = S mu (0: F = mu, zeroth order) */
  int32_t method;           /* pp_method (default PP_FOLDED) */
  int32_t contour_nodes;    /* PP_RIESZ: quadrature nodes on the upper half circle, 2n in all
                               (default 6, at most 32); the filter on a root at x = (omega -
                               omega0) / radius is 1 / (1 + x^(2n)) */
  double contour_tol;       /* PP_RIESZ: relative residual at which the shifted solves of the
                               first cycle stop (default 1e-4); later cycles stop at a tenth of
                               the window's worst residual, down to tol / 10 */
  int32_t contour_maxit;    /* PP_RIESZ: iteration cap of each shifted solve (default 500) */
  int32_t pass_vectors;     /* window solves: most particle-hole vectors per product pass (0,
                               the default: as many as the windows request at once, fewer when
                               their product workspaces would not fit the budget); a larger
                               request runs as several passes of equal size, each of which
                               rebuilds the amplitude strips when they are not stored */
} pp_options;

#define PP_MAX_ROOTS 64

typedef struct {
  int32_t cycles;               /* restart cycles used */
  int32_t basis;                /* final subspace size */
  int64_t products;             /* particle-hole vectors multiplied by (A, B, S) */
  int32_t n_roots;
  int32_t converged[PP_MAX_ROOTS];
  double residual[PP_MAX_ROOTS];  /* FP64 |(M - theta Sigma) y| / |y| per returned root */
  double seconds;               /* wall time of the solve */
  double sigma_seconds;         /* time inside the product kernels (device events) */
  double sigma_flops;           /* algorithmic flops of those products */
} pp_solve_info;

/* Fills *opt with the defaults documented above. */
void pp_default_options(pp_options* opt);

/* Copies the system to the device and builds what every product needs: layouts
 * of the DF factors, the Jacobi diagonal and, at order 2, the MP2 intermediates
 * (occupied/virtual MP2 density and energy-weighted density, the ring
 * intermediate Lambda_P,ia = sum_kc tau_ik^ac B_P,kc) from amplitude strips.
 * Returns PP_EINVAL for bad sizes or non-finite inputs, PP_ENOMEM when the
 * footprint exceeds opt->hbm_budget, PP_EDEVICE on a HIP error.  *out is NULL
 * on failure.  opt may be NULL (defaults). */
pp_status pp_setup(const pp_system* sys, const pp_options* opt, pp_handle** out);

/* out = M X (or Sigma X with PP_APPLY_METRIC) for m 2N-vectors.  X and out are
 * [m][2][n_occ][n_vir]; order (0..2) must not exceed the setup order.  The
 * contractions run in FP64, or with PP_REDUCED in the handle's reduced precision.
 * Synchronous, unless PP_ASYNC (which needs
 * PP_DEVICE_PTRS): the call then returns once the work is enqueued on the
 * handle's stream (opt->stream, or the stream the handle owns).  X must stay
 * unchanged and out unread until that work is done: work the caller orders after
 * it on opt->stream, pp_sync, or any later call on the handle (each waits for it
 * first).  Asynchronous calls keep their staging buffers (4 * 2m * N doubles for
 * the largest m so far) in the handle until pp_destroy. */
pp_status pp_sigma(pp_handle* h, int32_t order, int32_t m, const double* X, double* out, uint32_t flags);

/* The product of pp_sigma issued as n_parts calls, for passes too long to issue at
 * once: at second order the amplitudes are rebuilt in occupied strips in every pass (the
 * matrix-free product of the second-order equations), and at n_occ = 256, n_vir = 1024,
 * n_aux = 4096 one pass over 16 vectors is about 1e16 flops.  Part p multiplies the
 * amplitude strips of occupied rows [n_occ p / n_parts, n_occ (p + 1) / n_parts); part 0
 * also runs every contraction that does not depend on the strips (the first-order terms,
 * G = V B^vv - B^oo V, the delta-type second-order terms; with stored amplitudes the whole
 * amplitude contraction), and the last part the final combination, after which out holds
 * M X (or Sigma X).  Call parts 0 .. n_parts - 1 in order with the arguments of part 0;
 * X must stay unchanged and out unread until the last part is done.  The handle keeps
 * the pass's intermediates and staging (4 * 2m * N doubles) between parts and frees them
 * after the last.  Flags as pp_sigma (PP_ASYNC: each part returns once enqueued).
 * PP_EINVAL for n_parts outside 1..n_occ, a part out of order or with other arguments, or
 * a part after another product ran on the handle (the pass must start again at part 0);
 * otherwise as pp_sigma. */
pp_status pp_sigma_part(pp_handle* h, int32_t order, int32_t m, const double* X, double* out, uint32_t flags,
                        int32_t part, int32_t n_parts);

/* Waits until every product enqueued on the handle with PP_ASYNC is done. */
pp_status pp_sync(pp_handle* h);

/* pp_sigma for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same product,
 * same kernels and result, on device pointers only (PP_DEVICE_PTRS required), with the
 * staging of the trial and product vectors in a fixed scratch array of the library
 * (64 MiB per GPU, held until the process ends) and no timing events (the handle's
 * stats do not count these products).  It calls no allocating routine: the handle's
 * product workspace must already hold 2m vectors at the requested precision (an earlier
 * pp_sigma or window solve with at least m vectors on the handle grows it).  Every call
 * on one GPU shares that GPU's scratch array, so calls that overlap on one GPU (other
 * threads, other handles, PP_ASYNC calls not yet finished) race; with PP_ASYNC the
 * scratch stays in use until the work is done.  Errors: PP_EINVAL for host pointers,
 * 4 * 2m * N > 8 Mi doubles, or a workspace not yet reserved; otherwise as pp_sigma. */
pp_status pp_sigma_static(pp_handle* h, int32_t order, int32_t m, const double* X, double* out, uint32_t flags);

/* Roots of M z = omega Sigma z nearest omega0 on the positive branch, at the
 * handle's setup order: energies[n_roots] ascending (Ha); vectors
 * [n_roots][2][n_occ][n_vir] with X^T S X - Y^T S Y = 1 (nullable); osc
 * [n_roots] dipole oscillator strengths f = (2/3) omega sum_x (sqrt(2) F^x.(X+Y))^2 with
 * F = mu (or F = S mu with opt->correlated_f)
 * (nullable; needs dip at setup); info (nullable).  1 <= n_roots <= min(64, N). */
pp_status pp_window_solve(pp_handle* h, double omega0, int32_t n_roots, double* energies, double* vectors,
                          double* osc, pp_solve_info* info);

/* Several windows of the same system in one call: the windows are solved
 * concurrently (one host thread and one HIP stream each for the subspace work) and
 * their products are merged into shared product passes, so one pass of the
 * amplitude contraction serves several windows (two fixed groups of windows
 * alternate passes, so one group's subspace work overlaps the other's products;
 * results are reproducible).  omega0[n_windows]; outputs are
 * window-major: energies[n_windows][n_roots], vectors[n_windows][n_roots][2][n_occ][n_vir]
 * (nullable), osc[n_windows][n_roots] (nullable), info[n_windows] (nullable; the
 * product time/flops fields hold the totals of the whole call).  Each window's
 * result equals its pp_window_solve result within the solver tolerance.
 * PP_ENOTCONV if any window stopped at max_cycles (all outputs written). */
pp_status pp_window_solve_batch(pp_handle* h, int32_t n_windows, const double* omega0, int32_t n_roots,
                                double* energies, double* vectors, double* osc, pp_solve_info* info);

/* Cumulative device-side accounting of the handle's products (every pp_sigma
 * and every product inside pp_window_solve), timed with HIP events on the
 * handle's stream.  "hhat" is the dominant contraction H = tau G of the
 * second-order B term (one GEMM per amplitude strip batch). */
typedef struct {
  double product_flops;     /* algorithmic flops of all products */
  double product_seconds;   /* device time of all products */
  int64_t product_vectors;  /* particle-hole vectors multiplied */
  double hhat_flops;        /* algorithmic flops of the H = tau G GEMMs */
  double hhat_seconds;      /* device time of those GEMMs (sum over launches) */
  int64_t hhat_launches;
} pp_stats;

/* Fills *st (synchronizes the handle's stream). */
pp_status pp_get_stats(pp_handle* h, pp_stats* st);
/* Zeroes the accounting. */
pp_status pp_reset_stats(pp_handle* h);

/* MP2 correlation energy sum tau_ij^ab (ia|jb) found during an order-2 setup (0 otherwise). */
double pp_mp2_energy(const pp_handle* h);

/* Device bytes owned by the handle. */
uint64_t pp_device_bytes(const pp_handle* h);

/* Frees every device allocation of the handle.  NULL is accepted. */
pp_status pp_destroy(pp_handle* h);

/* Excitonic density of states of the Discussion section: for each energy bin
 * [edges[b], edges[b+1]) the number of particle-hole pairs ia whose orbital-energy
 * difference eps_a - eps_i falls in it (counts[b]) and the sum of their squared
 * transition dipoles sum_x (mu^x_ia)^2 (mu2[b]; zero without dip).  edges[n_bins+1]
 * ascending (Ha), counts and mu2 [n_bins] (mu2 nullable); host pointers.  Computed
 * on the device from the handle's copies of eps and the dipoles. */
pp_status pp_exciton_dos(pp_handle* h, int32_t n_bins, const double* edges, double* counts, double* mu2);

/* Broadened absorption spectrum from window roots (Results section: the spectra are
 * the roots' oscillator strengths broadened in frequency): for each grid point w_g,
 *     out[g] = sum_k osc[k] * (eta/pi) / ((w_g - energies[k])^2 + eta^2)
 * (a Lorentzian of half width eta per root; its integral over w is osc[k]).  Host
 * pointers: energies[n], osc[n], omega[n_omega], out[n_omega]; computed on the current
 * HIP device (the arrays are copied there and back).  PP_EINVAL for n < 0, n_omega < 0,
 * eta <= 0, energies not positive, non-finite values or NULL arrays with positive sizes;
 * PP_EDEVICE on a HIP error. */
pp_status pp_spectrum(int32_t n, const double* energies, const double* osc, int32_t n_omega, const double* omega,
                      double eta, double* out);

/* The isotropic dipole polarization propagator (Theory section: the propagator in its
 * non-diagonal representation, eq. pp_adc, Pi = F^T (w Sigma - M)^-1 F for the pencil of
 * the generalized eigenvalue equation) assembled from window roots in its spectral form:
 *     Pi(w) = sum_k osc[k] / (2 energies[k]) [1 / (w - energies[k]) - 1 / (w + energies[k])]
 * at w = omega[g] + i eta, i.e. (1/3) sum_x F_x^T (w Sigma - M)^-1 F_x with
 * F_x = sqrt(2) [mu_x; mu_x] restricted to the given roots (each positive root with its
 * partner -energies[k] on the negative branch; osc as the window solves return them, so
 * F = S mu with opt->correlated_f).  Given every root, it equals the resolvent form;
 * -Im Pi is the absorption-like spectrum and -Pi(0) the static polarizability.  Host
 * pointers: energies[n] (> 0, Ha), osc[n], omega[n_omega] (Ha), re and im [n_omega];
 * eta >= 0 (Ha; 0 gives the real axis, infinite at a root).  Computed on the current HIP
 * device.  PP_EINVAL for negative sizes, energies not positive, eta < 0, non-finite
 * values or NULL arrays with positive sizes; PP_EDEVICE on a HIP error. */
pp_status pp_response(int32_t n, const double* energies, const double* osc, int32_t n_omega, const double* omega,
                      double eta, double* re, double* im);

/* ------------------------------------------------------------------------
 * Serving: a persistent request loop for window solves of differing systems.
 *
 * Not in the paper (which solves one system at a time); it serves many
 * (system, omega0, n_roots) requests on one GPU with continuous batching:
 *  - pp_server_submit copies the request's inputs to host memory owned by the
 *    server and returns at once; requests are admitted in arrival order as soon
 *    as their device footprint (inputs, second-order intermediates, amplitudes
 *    when stored, product workspaces, subspace) fits the server's HBM budget
 *    and a solve slot is free;
 *  - each admitted request is set up on its own stream while earlier requests
 *    keep solving; its B tensors and subspace stay resident until it retires;
 *  - the products of all requests that are solving are merged into shared
 *    passes: each contraction step of the product is issued for every request at
 *    once, its GEMMs (different shapes) merged into grouped matrix-core launches;
 *  - a request retires when its window has converged (or failed); its device
 *    memory is released and the next queued requests are admitted.
 * Each request's result equals that of pp_window_solve on its own handle with the
 * same options, within the solver tolerance.  The server object is thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct pp_server pp_server;

/* Result of one request.  The caller sets the output pointers (each nullable,
 * host memory of the sizes given) before pp_server_poll / pp_server_wait; the
 * remaining fields are written by the server. */
typedef struct {
  double* energies;        /* [n_roots] ascending (Ha) */
  double* vectors;         /* [n_roots][2][n_occ][n_vir], X^T S X - Y^T S Y = 1 */
  double* osc;             /* [n_roots] oscillator strengths (0 when the system had no dip) */
  int32_t n_roots;         /* roots written */
  int32_t status;          /* pp_status of the solve (PP_OK, PP_ENOTCONV, PP_ENOMEM, ...) */
  pp_solve_info info;
  double queued_seconds;   /* submit -> admission */
  double run_seconds;      /* admission -> retirement (setup + solve) */
  double latency_seconds;  /* submit -> retirement */
} pp_result;

typedef struct {
  int64_t submitted, completed, failed, queued, running;
  int32_t peak_running;
  double latency_p50, latency_p99;   /* submit -> retirement over completed requests (s) */
  double queued_p50, queued_p99;     /* submit -> admission (s) */
  double solves_per_second;          /* completed / (last retirement - first submission) */
  int64_t passes;                    /* merged product passes */
  double mean_requests_per_pass;
  double product_flops;              /* algorithmic flops of all passes */
  double product_seconds;            /* device time of all passes (events on the pass stream) */
  uint64_t budget_bytes, reserved_bytes, peak_reserved_bytes;
  int64_t grouped_launches;          /* GEMM launches that served several requests at once */
} pp_server_stats;

/* opt: options applied to every request (NULL: defaults; hbm_budget, stream and
 * store_amplitudes are chosen per request by the server).  hbm_budget: device
 * bytes all admitted requests may hold together (0: 85% of free device memory).
 * max_active: requests solving at once (0: 8; at most 8). */
pp_status pp_server_create(const pp_options* opt, uint64_t hbm_budget, int32_t max_active, pp_server** out);

/* Queues a window solve of 'sys' (order 1 or 2; host arrays, copied before the
 * call returns).  PP_ENOMEM when its footprint alone exceeds the budget (nothing
 * queued), PP_EINVAL for bad sizes, non-finite inputs or device pointers. */
pp_status pp_server_submit(pp_server* srv, const pp_system* sys, double omega0, int32_t n_roots, uint64_t* req_id);

/* Device bytes the server would reserve for this request (its admission
 * footprint: an upper bound of what its setup, product workspace and subspace
 * allocate); 0 for invalid arguments.  Only the sizes and order of sys are read. */
uint64_t pp_server_request_bytes(const pp_server* srv, const pp_system* sys, int32_t n_roots);

/* Delivers a finished request's result into *res and forgets the request
 * (a second poll/wait of the same id returns PP_EINVAL).  Returns PP_EPENDING
 * (nothing written) while it is queued or running, otherwise the request's own
 * status (also in res->status). */
pp_status pp_server_poll(pp_server* srv, uint64_t req_id, pp_result* res);
/* As pp_server_poll, blocking until the request has finished. */
pp_status pp_server_wait(pp_server* srv, uint64_t req_id, pp_result* res);

/* Counters and latency percentiles since creation (or the last reset). */
pp_status pp_server_stats_get(pp_server* srv, pp_server_stats* st);
pp_status pp_server_stats_reset(pp_server* srv);

/* Finishes the running requests, drops the queued ones and frees everything. */
pp_status pp_server_destroy(pp_server* srv);

/* Last error message of the server (submit-time errors). */
const char* pp_server_last_error(const pp_server* srv);

const char* pp_status_string(pp_status s);
/* Last error message of the handle (NULL handle: last error, in this thread, of a call that
   takes no handle: pp_setup, pp_spectrum and the handle-less test hooks). */
const char* pp_last_error(const pp_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* PPWIN_H */
