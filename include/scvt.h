/*
 * scvt.h -- C ABI of libscvt.so: the per-iteration hot path of the
 * Lloyd-preconditioned LBFGS construction of spherical centroidal Voronoi
 * tessellations (Yang, Gunzburger & Ju, "Fast spherical centroidal Voronoi
 * mesh generation: a Lloyd-preconditioned LBFGS method in parallel").
 *
 * Problem (section 2.1): given generators Z = {z_i} on the unit sphere and a
 * density rho > 0, minimise the CCVT energy
 *     F(Z) = sum_i int_{V_i} |y - z_i|^2 rho(y) dsigma(y)
 * over the spherical Voronoi cells V_i of Z (eq. viInS, Euclidean metric).
 * One iteration (section 3.1 and the parallel algorithm of section 3.3 on a
 * single domain):
 *   1. Voronoi cells of Z (cube-map bucketing, bisector clipping with a
 *      security-radius certificate, sequential fallback);
 *   2. per cell: m_i = int rho, mu_i = int y rho (the paper's c_i),
 *      e_i = int |y - z_i|^2 rho  (fan triangles, geodesic subdivision,
 *      a triangle rule (7 points by default) through the radial-projection
 *      Jacobian);
 *   3. g_i = 2 (mu_i . z_i) z_i - 2 mu_i   (tangential gradient),
 *      h_i = 1 / (2 mu_i . z_i)            (spherical Lloyd preconditioner),
 *      l_i = mu_i/|mu_i| - z_i             (Lloyd step);
 *   4. LBFGS two-loop with the initial inverse Hessian diag(h) (section
 *      2.2.2 with eq. precStep);
 *   5. Armijo backtracking from alpha = 1 (the Lloyd step length), trial
 *      points projected back to the sphere; the pair (s, y) is stored when
 *      y.s > curv_eps |y||s|; at most M pairs are kept (section 4: M = 7).
 *
 * Conventions for every call:
 *   - Arrays of points are row-major n x 3 doubles (x, y, z per generator).
 *   - A pointer flagged "on_device" is a HIP device pointer on the current
 *     device; otherwise host memory.  The caller owns every buffer it passes;
 *     the library copies inputs and never returns memory it allocated.
 *   - Every call returns an int: 0 = success, > 0 = informational status,
 *     < 0 = error (see SCVT_E_*).  No C++ exception crosses the ABI.
 *   - A handle is not thread-safe; separate handles are independent.
 *   - All device work is ordered on the stream given in scvt_config
 *     (NULL: the library creates its own stream); calls return after the
 *     results they report are complete.
 */
#ifndef SCVT_H
#define SCVT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status and error codes */
#define SCVT_OK 0
#define SCVT_NOT_CONVERGED 1   /* scvt_solve stopped at max_iter */
#define SCVT_PENDING 2         /* serving: request not finished yet */
#define SCVT_E_INVALID -1      /* bad argument (n < 4, non-finite input, ...) */
#define SCVT_E_OOM -2          /* device allocation failed or over budget, or a host
                                  allocation failed (no C++ exception leaves a call) */
#define SCVT_E_DEGENERATE -3   /* duplicate or zero generators */
#define SCVT_E_CERT -4         /* a Voronoi cell could not be built */
#define SCVT_E_LINESEARCH -5   /* no sufficient decrease along the direction, and the
                                  Lloyd step taken instead raised F beyond the
                                  evaluation's rounding, max(ls_noise, 1e-13) |F|
                                  (section 2.2.1: it lowers the exact energy); the
                                  generators stay at the last iterate, the LBFGS
                                  history is cleared */
#define SCVT_E_NUMERIC -6      /* NaN, or mu_i . z_i <= 0 (h undefined) */
#define SCVT_E_HIP -7          /* a HIP runtime call failed */

typedef struct scvt_handle scvt_handle;

typedef enum { SCVT_FP64 = 0, SCVT_MIXED = 1 } scvt_precision;

/* Optimiser (section 2.2):
 *   SCVT_METHOD_PLBFGS -- LBFGS with the Lloyd preconditioner diag(h) as the
 *                         initial inverse Hessian (section 3.1), the default;
 *   SCVT_METHOD_LLOYD  -- Lloyd's iteration (section 2.2.1): z <- mu/|mu| for
 *                         every generator, no line search, no history;
 *   SCVT_METHOD_LBFGS  -- plain LBFGS with gamma_n I, gamma_n = y.s / y.y of the
 *                         newest stored pair (section 2.2.2; the identity while
 *                         no pair is stored), same line search and history. */
typedef enum { SCVT_METHOD_PLBFGS = 0, SCVT_METHOD_LLOYD = 1, SCVT_METHOD_LBFGS = 2 } scvt_method;

typedef enum {
  SCVT_RHO_CONST = 0, /* rho = 1 */
  SCVT_RHO_TANH = 1,  /* rho = gamma + sum_k amp_k (tanh((beta_k - d_k)/alpha_k) + 1)/2 */
  SCVT_RHO_X3 = 2,    /* rho = (1 - gamma) z^4 + gamma */
  SCVT_RHO_X16 = 3    /* tanh bump over the anisotropic distance of section 4 */
} scvt_rho_kind;

/* Density of section 4.  For SCVT_RHO_TANH, d_k = |y - xc_k| (chord) or the
 * geodesic angle when geodesic != 0; nbumps is 1 or 2.  The printed
 * prefactor 1/(2(1-gamma)) is read as (1-gamma)/2: pass amp = 1 - gamma for
 * the paper's single bump.  SCVT_RHO_X16 uses xc[0], beta[0], alpha[0],
 * amp[0], gamma, w_lon, w_lat. */
typedef struct {
  int32_t kind;
  int32_t geodesic;
  int32_t nbumps;
  int32_t reserved;
  double xc[2][3];
  double beta[2];
  double alpha[2];
  double amp[2];
  double gamma;
  double w_lon, w_lat;
} scvt_density;

typedef struct {
  int64_t n;            /* number of generators (4 .. 2^28) */
  int32_t m_hist;       /* M, stored LBFGS pairs (0 = Lloyd iteration) */
  int32_t precision;    /* scvt_precision */
  scvt_density rho;
  int32_t quad_levels;  /* geodesic subdivision levels per fan triangle (0..3, default 2) */
  int32_t ls_max_evals; /* energy evaluations per line search (default 10) */
  double ls_c1;         /* Armijo constant (default 1e-4) */
  double curv_eps;      /* store (s,y) only if y.s > curv_eps |y||s| (default 1e-10) */
  double ls_noise;      /* Armijo allowance: accept F' <= F + c1 alpha g.q + ls_noise |F|;
                           < 0 = automatic: 0 for FP64, 1e-8 for the mixed path, whose FP32
                           quadrature leaves ~1e-9 relative noise in energy differences */
  int32_t keep_cells;   /* 1: keep a copy of every cell for scvt_get_cells */
  int32_t method;       /* scvt_method (default SCVT_METHOD_PLBFGS) */
  int32_t quad_rule;    /* points of the triangle rule: 7 (Radon, degree 5; default), or the
                           conical product rules of the sizes section 4.1 uses: 4 (degree 3),
                           9 (degree 5) */
  int32_t k_max;        /* > 0: at most k_max candidates per cell in the certified passes
                           (16, 32 and 64 otherwise); cells needing more go on to the next
                           pass and finally to the sequential clipper, which builds the same
                           cell (a test knob for the fallback path; 0 = default) */
  void* hip_stream;     /* hipStream_t to order work on, or NULL */
} scvt_config;

/* Per-iteration record; the columns of the paper's tables (section 4). */
typedef struct {
  int64_t iter;         /* iterations done */
  int64_t n_evals;      /* energy evaluations done (incl. the initial one) */
  double F;             /* energy at the current generators */
  double grad_norm2;    /* |g|_2 */
  double step_inf;      /* max_i,k |l_ik| (Lloyd step, the stopping measure) */
  double alpha;         /* accepted step length of the last iteration */
  int64_t n_fallback;   /* cells built by the fallback clipper, last evaluation */
  int64_t n_degenerate; /* cells with a predicate inside its error bound */
  int32_t status;       /* last return code */
  int32_t hist_len;     /* stored pairs */
  int64_t n_lloyd_fallback; /* iterations that took the Lloyd step after the
                               line search found no sufficient decrease */
  int64_t n_wide[2];    /* cells the 8-lane pass handed to the 16-lane pass,
                           and that pass to the 64-lane one, last evaluation */
} scvt_info;

/* The per-iteration records: a handle keeps the last SCVT_RECORD_RING of
 * them -- the initial evaluation's (iter 0) and one after every iteration, as
 * scvt_step would return them (status SCVT_OK) -- the columns of the paper's
 * iteration histories (section 4: F and |grad F| against iterations).  out:
 * host array of max records (caller-owned), filled oldest first with the last
 * min(max, kept) records; *count (optional) receives how many.  Errors:
 * SCVT_E_INVALID (NULL handle, max < 0, or out NULL with max > 0). */
#define SCVT_RECORD_RING 4096
int scvt_get_records(scvt_handle* h, int64_t max, scvt_info* out, int64_t* count);

/* Fill *cfg with defaults for n generators (section 4's settings: M = 7,
 * ten energy evaluations per line search): FP64, rho = 1,
 * 2 subdivision levels, 10 evaluations per line search, c1 = 1e-4,
 * curv_eps = 1e-10, automatic ls_noise, no cell copy, NULL stream. */
int scvt_config_init(scvt_config* cfg, int64_t n);

/* Create a solver for the problem of section 2.1 (generators on the unit
 * sphere, density rho, CCVT energy).  z0: n x 3 (host, or device if
 * z0_on_device); rows are normalised to the unit sphere.  Allocates all device state, builds the
 * cells of z0 and evaluates F, g, h and the Lloyd step (iteration 0 ready).
 * Errors: SCVT_E_INVALID (n < 4, bad config, non-finite z0), SCVT_E_OOM,
 * SCVT_E_DEGENERATE (zero row), SCVT_E_CERT, SCVT_E_NUMERIC, SCVT_E_HIP.
 * *out is NULL on error. */
int scvt_create(const scvt_config* cfg, const double* z0, int z0_on_device, scvt_handle** out);

/* One iteration of the configured method (section 3.1 with the two-loop
 * recursion of section 2.2.2).  P-LBFGS and LBFGS: two-loop
 * direction, descent check with reset to the history-free direction, Armijo
 * line search, history update; if the line search finds no sufficient
 * decrease in ls_max_evals evaluations, the history is cleared and the Lloyd
 * step (alpha = 1) is taken, which decreases F in exact arithmetic (section
 * 2.2.1); SCVT_E_LINESEARCH if it does not.  Lloyd: the Lloyd step, one
 * evaluation.  info may be NULL. */
int scvt_step(scvt_handle* h, scvt_info* info);

/* Iterate until step_inf < tol_step_inf or max_iter iterations in total
 * (the stopping test on the generators' movement, section 3.3).
 * Returns SCVT_OK when converged, SCVT_NOT_CONVERGED at the cap, or an error. */
int scvt_solve(scvt_handle* h, int64_t max_iter, double tol_step_inf, scvt_info* info);

/* scvt_solve with the stopping tests of the paper's method comparison
 * (section 4.1): stop when max |l_ik| < step_tol, or (quasi-Newton methods
 * only) |g|_2 / F <= grad_rel_tol, or |F_prev - F| / F_prev < f_rel_tol, or
 * after max_iter iterations (SCVT_NOT_CONVERGED).  A tolerance <= 0 disables
 * its test. */
int scvt_solve_rel(scvt_handle* h, int64_t max_iter, double step_tol, double grad_rel_tol,
                   double f_rel_tol, scvt_info* info);

/* Cached results at the current generators (no recomputation): the CCVT
 * energy F and the mass centroids of section 2.1: F, and
 * optionally per cell mass (n), centroid mu_i/m_i (n x 3) and energy e_i (n).
 * Any output pointer may be NULL. */
int scvt_energy(scvt_handle* h, double* F, double* mass, double* centroid, double* e_cell,
                int out_on_device);

/* Current generators, n x 3 (the iterate z of section 3.1). */
int scvt_get_generators(scvt_handle* h, double* z, int on_device);

/* Per-generator vectors at the current generators (section 3.1's gradient,
 * preconditioner and Lloyd step; parity and debugging):
 * which = 0 gradient g (n x 3), 1 preconditioner h (n), 2 Lloyd step l
 * (n x 3), 3 first moment mu (n x 3), 4 the last search direction q (n x 3),
 * 5 cell circumradius (n). */
int scvt_get_vectors(scvt_handle* h, int which, double* out, int on_device);

/* Compute the P-LBFGS direction (the two-loop recursion of section 2.2.2
 * with the initial inverse Hessian of section 3.1) at the current state into
 * out (n x 3),
 * without stepping; *gq receives g . q (may be NULL). */
int scvt_direction(scvt_handle* h, double* out, int on_device, double* gq);

/* Voronoi cells at the current generators (eq. viInS of section 2.1;
 * requires keep_cells = 1).
 * max_deg must be 32.  nbr: n x 32 neighbour ids sorted ascending, -1 padded;
 * deg: n; verts: n x 32 x 6, edge k of cell i runs counter-clockwise (seen
 * from outside) from verts[i][k][0:3] to verts[i][k][3:6] on the bisector of
 * i and nbr[i][k]; flags: n, bit 1 fallback-built, 2 near-degenerate,
 * 4 error, 8 brute-force search.  Any output may be NULL.  Host memory. */
int scvt_get_cells(scvt_handle* h, int32_t max_deg, int32_t* nbr, int32_t* deg, double* verts,
                   uint8_t* flags);

/* Number of generators of a handle (n of section 2.1). */
int scvt_num_generators(scvt_handle* h, int64_t* n);

/* Bisection step of the optimisation-bisection initialisation (section 3.3;
 * section 4.3 refines a converged 2,562-generator SCVT up to 655,362): the
 * current generators followed by the normalised midpoint of every Delaunay
 * edge (i, j) -- generators whose cells share a Voronoi edge -- ordered by i,
 * then j (i < j).  A spherical triangulation has 3n - 6 edges, so n becomes
 * 4n - 6.  *n_out receives the new count; z_out (n_out x 3, host, or device
 * when on_device) may be NULL to query it.  Uses temporary device memory;
 * the handle's state is unchanged. */
int scvt_refine(scvt_handle* h, double* z_out, int on_device, int64_t* n_out);

/* The optimisation-bisection driver: create a handle from z0 (cfg0->n
 * generators), solve it (scvt_solve with max_iter and tol), then `levels`
 * times refine it (scvt_refine) into a new handle with the same settings
 * and solve again.  infos (levels + 1 entries, may be NULL) receives each
 * level's final record; *out the last level's handle (caller destroys).
 * Returns SCVT_OK, SCVT_NOT_CONVERGED if the last level stopped at max_iter,
 * or an error (then *out is NULL). */
int scvt_multilevel(const scvt_config* cfg0, const double* z0, int z0_on_device, int levels,
                    int64_t max_iter, double tol, scvt_info* infos, scvt_handle** out);

/* scvt_refine for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same result, written to the device buffer z_out (n_out x 3; NULL to query
 * *n_out only), with no hipMalloc or hipFree.  Its temporary buffers live in
 * one static device array per GPU (96 MiB, held by every GPU the library
 * runs on until the process ends), enough for SCVT_REFINE_NOALLOC_MAX_N
 * generators (the paper's largest bisection input, section 4.3); larger
 * handles return SCVT_E_OOM.  Calls on one GPU share the array: calls that
 * overlap in time on one GPU race (serialise them); nothing in it has to
 * start cleared.  Uses the handle's own buffers and stream otherwise. */
#define SCVT_REFINE_NOALLOC_MAX_N 655362
int scvt_refine_noalloc(scvt_handle* h, double* z_out, int64_t* n_out);

/* Mesh export and quality (sections 3.3 and 4) at the current generators:
 * the Delaunay triangles, each once as (i, j, k) with i its smallest index,
 * counter-clockwise seen from outside, ordered by i then j (2n - 4 of them
 * for points in general position); cellQ = min / max edge of every Voronoi
 * cell; triQ = (a+b-c)(b+c-a)(c+a-b)/(abc) of every triangle, in the order of
 * the list.  Lengths are chords.  *ntri receives the triangle count; tri
 * (ntri x 3), cell_q (n) and tri_q (ntri) are host buffers and may be NULL
 * (call once with all NULL to size tri and tri_q).  Uses temporary device
 * memory; the handle's state is unchanged. */
int scvt_mesh(scvt_handle* h, int32_t* tri, int64_t* ntri, double* cell_q, double* tri_q);

/* Checkpoint of the iteration of section 3.1 (its state is the generators
 * and the LBFGS pairs of section 2.2.2): serialise (Z, history ring,
 * counters) into buf.  With buf ==
 * NULL, *bytes receives the size needed.  scvt_set_state restores a state
 * produced by a handle with the same n and M and re-evaluates at Z. */
int scvt_get_state(scvt_handle* h, void* buf, size_t* bytes);
int scvt_set_state(scvt_handle* h, const void* buf, size_t bytes);

/* Kernel timing of the iteration's steps (section 3.1's evaluation and
 * direction; HIP events on the handle's stream, enabled by
 * scvt_set_timing: 0 off, 1 every timer below, 2 only the quadrature
 * kernel's, two events per evaluation): kernel 0 = certified cell geometry
 * kernel, 1 = fallback
 * clipper, 2 = grid build, 3 = two-loop passes, 4 = whole evaluation,
 * 5 = cell quadrature kernel, 6 = list passes of the certified geometry
 * (cells needing more candidates than the main geometry kernel holds).
 * Returns accumulated milliseconds and launch count since enabling. */
int scvt_set_timing(scvt_handle* h, int enable);
int scvt_kernel_time(scvt_handle* h, int kernel, double* total_ms, int64_t* launches);

/* Release a handle and all its device state (NULL is ignored). */
void scvt_destroy(scvt_handle* h);
/* Text of a status code (the SCVT_* values above). */
const char* scvt_strerror(int code);

/* Device memory a handle with this configuration allocates (bytes): the
 * generators, cells and LBFGS history of section 3.1 for n and M. */
int scvt_footprint(const scvt_config* cfg, size_t* bytes);

/* ------------------------------------------------------------- serving --
 * Continuous batching of solves (north of the per-iteration path of
 * section 3.1; the paper has no serving): requests of any size and tanh or
 * other density are submitted at any time.  A request is admitted when one
 * of max_slots slots is free and its footprint (scvt_footprint) fits in a
 * free range of the server's device arena of hbm_budget bytes, first come
 * first served; its generators, cells and LBFGS history then live in that
 * range until it finishes.  One driver thread runs rounds on `stream`: every
 * admitted request's next evaluation (with its direction passes and trial
 * point) is issued as one segmented launch per kernel over all of them,
 * followed by one gather of their scalars and one synchronisation; each
 * request then takes its own line-search and history decisions (those of
 * scvt_solve), until step_inf < tol or max_iter iterations.  Requests join
 * and leave at round boundaries.  A request's result does not depend on the
 * other requests (every kernel computes a request's cells and reductions as
 * its own launch would).
 * Served: P-LBFGS with m_hist <= 16 (other methods: SCVT_E_INVALID).  All
 * device and pinned memory is allocated by scvt_server_create; nothing is
 * allocated per request.  The server uses the device current at creation;
 * stream NULL: its own.  Submit copies z0 (host, n x 3); cfg->hip_stream is
 * ignored.  Errors: SCVT_E_INVALID, SCVT_E_OOM (footprint above the whole
 * budget, or the budget cannot be allocated; also a failed host allocation:
 * in the driver thread it fails every admitted and waiting request and
 * every later submission with SCVT_E_OOM). */
typedef struct scvt_server scvt_server;
int scvt_server_create(size_t hbm_budget, int max_slots, void* stream, scvt_server** out);
int scvt_server_submit(scvt_server* s, const scvt_config* cfg, const double* z0, double tol,
                       int64_t max_iter, int64_t* req_id);
/* SCVT_PENDING while waiting or running; otherwise the request's final
 * status (SCVT_OK, SCVT_NOT_CONVERGED or an error), with the final
 * generators in z_out (n x 3 host, may be NULL), its record in info and
 * times[0..2] = submission, admission and completion (seconds, steady
 * clock), each output optional. */
int scvt_server_poll(scvt_server* s, int64_t req_id, double* z_out, scvt_info* info,
                     double* times);
/* Forget a finished request (frees its host copy of the result). */
int scvt_server_release(scvt_server* s, int64_t req_id);
/* Queue depth, running requests and device bytes held by them. */
int scvt_server_stats(scvt_server* s, int64_t* waiting, int64_t* running, size_t* bytes_used);
/* Drops waiting requests, waits for running ones, frees everything. */
void scvt_server_destroy(scvt_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SCVT_H */
