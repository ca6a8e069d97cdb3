/*
 * hfmm.h -- C ABI of the MI355X Helmholtz FMM / BIE / GMRES library.
 *
 * The library computes the dense matrix-vector product of the Helmholtz
 * single-layer kernel G(x, y) = e^{ikR} / (4 pi R), R = |x - y| (eq. (6) of
 * arXiv 1803.09948) with a spherical-harmonic fast multipole method over an
 * adaptive Morton-ordered octree (Sec. 2.3: upward P2M/M2M, traversal M2L/P2P,
 * downward L2L/L2P), and solves the sound-soft boundary integral equation
 * eq. (7) with restarted GMRES (Sec. 5.1, Sec. 6.4).  The tree build and the
 * dual tree traversal (Sec. 3.1, Sec. 3.2) are setup and run in host C++;
 * every step of the product and of GMRES runs as a hand-written HIP kernel
 * for gfx950.
 *
 * Conventions shared by all calls
 *  - Return value: HFMM_OK (0) on success, a negative code on error, or
 *    HFMM_ENOTCONV (1) as a warning from the solver.  No C++ exception ever
 *    crosses this boundary.  On error hfmm_last_error() returns a message for
 *    the calling thread; no output has been written unless stated.
 *  - "_host" pointers are host memory owned by the caller and only read
 *    during the call.  "_dev" pointers are device memory on the current HIP
 *    device, owned by the caller, and accessed in stream order on `stream`
 *    (hipStream_t passed as void*; NULL is the default stream).
 *  - Complex vectors are interleaved (re, im): float2 = 8 bytes, double2 =
 *    16 bytes per entry.  Vectors are always in the caller's original point
 *    (or panel) order; the Morton order is internal.
 *  - Expansion order P counts degrees 0..P-1 (P^2 coefficients; the text
 *    after eq. (14)).  1 <= P <= 16.
 *  - A tree handle owns its device memory.  Building a handle touches no
 *    device memory; the bodies are uploaded and the operators of a (k, P)
 *    are built on the device when that (k, P) is first prepared (explicitly
 *    by hfmm_prepare, or implicitly by the first product or solve); a
 *    product that reuses a prepared (k, P) allocates nothing; GMRES adds its
 *    Krylov workspace on the first solve with a given restart.
 *    hfmm_tree_plan reports every one of these sizes beforehand, on the
 *    host.  A handle keeps one set of product buffers (strengths, sorted
 *    outputs, expansions, staging), so calls on one handle must not overlap:
 *    from several host threads or on several streams they need external
 *    serialisation (a stream-ordered wait between them suffices).
 */
#ifndef HFMM_H
#define HFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HFMM_OK = 0,
  HFMM_ENOTCONV = 1,   /* GMRES hit maxit: x holds the last iterate, info filled */
  HFMM_EINVAL = -1,    /* bad argument; nothing was done */
  HFMM_ENOMEM = -2,    /* device or host allocation failed */
  HFMM_EHIP = -3,      /* a HIP call failed; message in hfmm_last_error() */
  HFMM_EINTERNAL = -4
};

typedef struct hfmm_tree hfmm_tree;

/* Tree / traversal options (the paper leaves these unspecified, Sec. 3.2). */
typedef struct {
  int32_t ncrit;     /* a cell with more than ncrit sources splits (default 64) */
  int32_t max_level; /* deepest level (default 20, at most 20) */
  double theta;      /* acceptance: 3 (sA+sB)^2 < theta^2 D2 (default 0.5) */
  double kappa;      /* and k * cell side <= kappa; < 0 means 0.4 * P (default -1) */
  double eta;        /* BIE near pattern |c_i - c_j| < eta h_j (default 2) */
  int32_t near_levels; /* BIE near integrals: 4^near_levels sub-triangles (default 3) */
  int32_t near_order;  /* BIE near integrals: n x n collapsed Gauss rule (default 6) */
  int32_t stage_mb;    /* M2L staging budget in MiB (default 32768; <= 0: default): larger
                          problems run the M2L in segments of targets whose staging fits;
                          the staging then holds two segments, so that one segment's
                          reduction overlaps the next segment's M2L */
  int32_t bie_treatment; /* BIE singular-integral treatment: 0 self + near corrections
                            (default), 1 self-panel integral only, 2 none (the 3-point rule
                            everywhere, the listing without its near branch) */
  double k_imag;        /* imaginary part of the wavenumber: every call on the handle uses
                            k + i k_imag (damped waves, the imaginary wavenumber of the P2P
                            listing of Sec. 3.1); >= 0, default 0.  The tree rules use
                            |k + i k_imag|; the plane wave becomes exp(i (k + i k_imag) d.x).
                            The FP64 variant (hfmm_matvec64) takes k_imag = 0 only */
  int32_t reserved[4];
} hfmm_opts;

typedef struct {
  int64_t n_src, n_tgt;       /* bodies */
  int32_t n_cell, n_leaf, n_level;
  int32_t point_mode;         /* 1: sources = targets (plain matvec) */
  double centre[3], half;     /* root cube */
  int64_t n_m2l, n_p2p;       /* cell pairs of the traversal at (k, P) */
  int64_t p2p_body_pairs;     /* sum over P2P pairs of n_tgt * n_src */
  int64_t n_tables;           /* distinct M2L translation operators */
  int64_t n_near;             /* BIE near-correction nonzeros */
  int64_t device_bytes;       /* device memory held by the handle */
} hfmm_stats;

/* Sizes of a (k, P) plan, computed on the host before any device memory is
 * touched (hfmm_tree_plan).  Bytes are device bytes. */
typedef struct {
  int64_t n_src, n_tgt;       /* bodies */
  int32_t n_cell, n_leaf, n_level;  /* cells of the tree used at (k, P) */
  int32_t resident;           /* 1 when the (k, P) operators are already on the device */
  int64_t n_m2l, n_p2p;       /* traversal cell pairs */
  int64_t p2p_body_pairs;     /* sum over P2P pairs of n_tgt * n_src */
  int64_t n_tables;           /* distinct M2L translation operators */
  int64_t n_near;             /* BIE near-correction nonzeros */
  int64_t bytes_tree;         /* resident bodies, permutations, BIE geometry and near
                                 pattern, and the cells of the (k, P) tree */
  int64_t bytes_lists;        /* M2L pair records, P2P work and source intervals */
  int64_t bytes_expansions;   /* translation tables, multipole and local expansions
                                 M, L (2 x cells x P^2 complex64), M2L staging */
  int64_t bytes_corrections;  /* BIE near values and self terms at k (0 for points) */
  int64_t bytes_gmres;        /* GMRES(restart) workspace (0 for point handles) */
  int64_t bytes_total;        /* sum of the five above */
} hfmm_plan_info;

typedef struct {
  int32_t iters;       /* matrix-vector products inside Arnoldi steps */
  int32_t restarts;
  double resid_est;    /* Arnoldi estimate |g_{j+1}| / ||b|| at exit */
  double resid_true;   /* ||b - A x|| / ||b|| recomputed at exit */
  double seconds;
} hfmm_gmres_info;

/* Fills `opts` with the defaults above. */
int hfmm_default_opts(hfmm_opts* opts);

/* Point-mode tree over n points (sources = targets), Sec. 2.3 and Sec. 3.1.
 *  xyz_host: n x 3 float32, row-major (x0 y0 z0 x1 ...).
 *  opts: NULL for defaults.
 *  EINVAL: n < 1, non-finite coordinates, ncrit < 1, theta <= 0.
 *  On success *out is a new handle (free with hfmm_tree_free). */
int hfmm_build_tree(const float* xyz_host, int64_t n, const hfmm_opts* opts,
                    hfmm_tree** out);

/* BIE handle for a closed flat-triangle surface (eq. (7) discretised by
 * centroid collocation, Sec. 2.2): the unknown is one density value per
 * triangle; sources are 3 interior Gauss points per triangle (weight A/3),
 * targets are the centroids.  Near panels (|c_i - c_j| < eta h_j) get an
 * accurate panel integral and the diagonal the weakly singular self integral
 * (Sec. 2.2 and the near/self branches of the P2P listing in Sec. 3.1).
 *  verts_host: nv x 3 float64;  tris_host: nt x 3 int32 vertex indices.
 *  EINVAL: nv < 3, nt < 1, index out of range, degenerate triangle. */
int hfmm_build_bie(const double* verts_host, int64_t nv, const int32_t* tris_host,
                   int64_t nt, const hfmm_opts* opts, hfmm_tree** out);

/* BIE handle for a closed surface of curved six-node triangles, by the
 * locally corrected Nystrom method of Sec. 2.2 (eqs. (8)-(10)).
 *  Geometry: the quadratic map of the reference triangle through the nodes
 *    (v0, v1, v2, m01, m12, m20) of each element.
 *  Unknowns: six per element, at the points of the symmetric degree-4
 *    six-point rule (three near the corners, three near the edges, as in the
 *    dataset of Sec. 5), element-major.  The unknown is the density times
 *    the surface Jacobian at the point (eq. (8)).
 *  Matrix: far entries are the rule weight times G. The own element is
 *    integrated by a Duffy rule with an angular sinh map. Elements whose
 *    centroid lies within eta h of the target point use 4^near_levels
 *    sub-triangles with near_order^2 points each.
 *  Computed: corrections in FP64, near ones stored in complex64; self blocks
 *    are applied in FP64 by GMRES.
 *  nodes_host: nn x 3 float64; tri6_host: nt x 6 int32 node indices.
 *  Works with hfmm_matvec, hfmm_gmres_solve and hfmm_bie_plane_wave (at the
 *  points).
 *  EINVAL: nn < 6, nt < 1, index out of range, degenerate element. */
int hfmm_build_nystrom(const double* nodes_host, int64_t nn, const int32_t* tri6_host,
                       int64_t nt, const hfmm_opts* opts, hfmm_tree** out);

/* Points of a curved-element handle (host arrays of 6 nt entries, any may
 * be NULL): positions (x 3), rule weights (parametric, summing to 1/2 per
 * element) and surface Jacobians.  The density at point p is
 * unknown_p / jac_p.  EINVAL for other handles. */
int hfmm_nystrom_points(const hfmm_tree* tree, double* xyz_host, double* weight_host,
                        double* jac_host);

/* Builds (once) the traversal lists, translation operators and, for a BIE
 * handle, the near and self corrections for wavenumber k and order P, and
 * the execution state of a product: its work lists, its M2L launch shape
 * (the first call times each shape on this work; see hfmm_variant_count)
 * and a second stream with two events (the near field runs beside the far
 * field).  Afterwards hfmm_matvec on (k, P) allocates nothing.
 * Called implicitly by hfmm_matvec / hfmm_gmres_solve.  It allocates and
 * waits on `stream`, so it must not run while `stream` is being captured
 * into a graph.
 *  EINVAL: k <= 0 or non-finite, P outside [1, 16]. */
int hfmm_prepare(hfmm_tree* tree, double k, int32_t P, void* stream);

/* y = A x (Sec. 2.3; eq. (11) for a point handle, the collocation matrix of
 * eq. (7) for a BIE handle), FP32 arithmetic with FP32 accumulation.
 *  x_dev: complex64[n] (point handle) or complex64[nt] (BIE handle).
 *  y_dev: complex64, same length; must not alias x_dev.
 *  Point handle: y_i = sum_{j, R_ij > 0} x_j G(x_i, x_j) up to FMM truncation. */
int hfmm_matvec(hfmm_tree* tree, double k, int32_t P, const void* x_dev,
                void* y_dev, void* stream);

/* FP64 variant of hfmm_matvec for a point handle: the same tree, lists,
 * translation operators and P (eq. 12-14 truncated at P), every step in
 * FP64, so that its difference to hfmm_matvec is the FP32 rounding of the
 * product and its difference to the direct sum the truncation error.  A
 * precision reference, not a fast path (plain kernels; M2L accumulates with
 * FP64 atomics, so the last bits may vary between calls).
 *  x_dev, y_dev: complex128[n] device, caller order; must not alias.
 *  Allocates FP64 tables and expansions on first use for (k, P).
 *  EINVAL: BIE handle, NULL, k or P as for hfmm_matvec.  ENOMEM, EHIP. */
int hfmm_matvec64(hfmm_tree* tree, double k, int32_t P, const void* x_dev,
                  void* y_dev, void* stream);

/* Direct sum in FP64 on the device (eq. (11) with the kernel of eq. (6)):
 * y_i = sum_{j: R_ij > 0} q_j exp(i k R_ij) / (4 pi R_ij), R_ij = |t_i - s_j|.
 *  src_dev: float[n][3], q_dev: complex128[n], tgt_dev: float[m][3],
 *  y_dev: complex128[m]; all device memory owned by the caller.
 *  EINVAL: n or m negative, NULL pointers, k negative or non-finite. */
int hfmm_direct64(const float* src_dev, const void* q_dev, int64_t n,
                  const float* tgt_dev, int64_t m, double k, void* y_dev,
                  void* stream);

/* Restarted GMRES(restart) for A x = b on a BIE handle (Sec. 5.1: complex
 * GMRES, exit at a relative residual tol, Sec. 6.4).  The Arnoldi
 * orthogonalisation (two passes of classical Gram-Schmidt), the Givens
 * least-squares update and the self-panel diagonal run in FP64 on the
 * device; the FMM product in FP32.
 *  b_dev: complex128[nt];  x_dev: complex128[nt], in: initial guess, out: x.
 *  Returns HFMM_OK when ||b - A x|| / ||b|| <= tol, HFMM_ENOTCONV after maxit
 *  products (x then holds the last iterate).  EINVAL: tol <= 0, restart < 1,
 *  restart > 200, maxit < 1, point handle. */
int hfmm_gmres_solve(hfmm_tree* tree, double k, int32_t P, const void* b_dev,
                     void* x_dev, double tol, int32_t restart, int32_t maxit,
                     hfmm_gmres_info* info, void* stream);

/* hfmm_gmres_solve without device allocation, for callers that cannot
 * allocate at solve time (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same solver, kernels and result
 * bits; the Krylov workspace ((restart + 1) complex128 basis vectors of nt
 * entries plus work vectors and small arrays: ((restart + 4) x 16 + 8) x nt
 * bytes and a few KiB) lives in a static device array of 72 MiB that each device
 * holds for the life of the process.  Calls on one device share
 * that array: calls that overlap on one device race (serialise them); its
 * contents on entry do not matter.
 *  Requires (k, P) prepared on the handle (hfmm_prepare), since preparing
 *  allocates: EINVAL otherwise.  ENOMEM (nothing done) when the workspace
 *  exceeds 72 MiB (e.g. nt > 136,000 at restart 30).  Other arguments and
 *  results as hfmm_gmres_solve. */
int hfmm_gmres_solve_noalloc(hfmm_tree* tree, double k, int32_t P, const void* b_dev,
                             void* x_dev, double tol, int32_t restart, int32_t maxit,
                             hfmm_gmres_info* info, void* stream);

/* b_i = exp(i k d . c_i) at the centroids of a BIE handle (complex128[nt],
 * caller order), or at the points of a curved-element handle
 * (complex128[6 nt]): the incident plane wave of eq. (7).  dir_host: 3
 * doubles. */
int hfmm_bie_plane_wave(hfmm_tree* tree, double k, const double* dir_host,
                        void* b_dev, void* stream);

/* One fused launch sequence for `count` independent point-mode products
 * y_i = A_i x_i (each with its own tree and k; one P for all).  The work
 * lists of all instances are concatenated, so each phase (and each tree
 * level) is a single launch over every instance and uneven instances fill
 * the chip together; the sequence is captured once as a HIP graph (per set of
 * trees, k and P) and replayed on later calls.  Each result is bitwise
 * equal to hfmm_matvec on that instance alone: every phase sums in a fixed
 * order (the M2L through staging slots reduced per target).
 * trees, ks, Ps, xs_dev, ys_dev: arrays of length count.  EINVAL as for
 * hfmm_matvec, count < 1, differing P, a BIE handle, or a handle that appears
 * twice (its instances would share the handle's product buffers). */
int hfmm_batch_matvec(int32_t count, hfmm_tree* const* trees, const double* ks,
                      const int32_t* Ps, const void* const* xs_dev,
                      void* const* ys_dev, void* stream);

/* Host half of hfmm_prepare: builds the cells, traversal lists, operator
 * descriptors and work lists for (k, P) without touching the device, and
 * reports the exact device bytes the operator will take (plus the bodies if
 * not yet resident).  Safe to call for different handles from different
 * threads.  footprint_bytes may be NULL.  EINVAL as for hfmm_prepare. */
int hfmm_prepare_host(hfmm_tree* tree, double k, int32_t P, int64_t* footprint_bytes);

/* Plan of a (k, P) product and solve on the host (the admission question
 * of a matrix-free GMRES, Sec. 1 and Sec. 2.3): builds the tree used at
 * (k, P), the traversal lists and the work lists (as hfmm_prepare_host; kept
 * for the later device half), and reports counts and the device bytes of
 * each part.  Touches no device memory.  restart: the GMRES restart the
 * workspace is sized for (1..200 for BIE handles, 0 allowed for point
 * handles, whose bytes_gmres is 0).  The counts are those hfmm_tree_stats
 * reports after preparation; the bytes are what the library allocates.
 *  EINVAL: NULL, k or P as for hfmm_prepare, restart out of range. */
int hfmm_tree_plan(hfmm_tree* tree, double k, int32_t P, int32_t restart,
                   hfmm_plan_info* out);

/* ---- Continuous-batching solve server -----------------------------------
 * Serves many BIE solves at once.  Submitted solves wait in a queue; every
 * hfmm_server_step admits queued solves (first come, first served) while
 * fewer than max_active run and their device footprint fits the budget
 * (0 = no limit), then advances each running solve by one GMRES product: a
 * fused FMM launch sequence per expansion order P present among them, then
 * each solve's FP64 Arnoldi / residual work, and one host synchronisation
 * for all.  Solves join and leave at step boundaries; each result is
 * bitwise that of hfmm_gmres_solve on the same system (every accumulation
 * of the fused sequence has the order of the single product).  Handles, b
 * and x must stay valid until the solve is done; one solve per handle at a
 * time.  Not thread-safe: drive a server from one thread. */
typedef struct hfmm_server hfmm_server;

int hfmm_server_create(int64_t hbm_budget_bytes, int32_t max_active, hfmm_server** out);
/* Early-stop policy (failure detection for solves that cannot converge in
 * reasonable time; off by default).  At each restart boundary, after the
 * true residual is known, a solve stops in state 4 when
 *  - stall_restarts > 0 and its true relative residual is not below
 *    stall_factor times its value stall_restarts restarts earlier, or
 *  - max_seconds > 0 and it has been active longer than max_seconds.
 * x then holds the last iterate and info its residuals.
 *  EINVAL: stall_restarts < 0, stall_factor outside (0, 1], max_seconds < 0. */
int hfmm_server_set_limits(hfmm_server* server, int32_t stall_restarts, double stall_factor,
                           double max_seconds);
/* Queues a solve; *ticket identifies it, *footprint_bytes (may be NULL) is
 * the device memory it will hold while active.  ENOMEM if it can never fit. */
int hfmm_server_submit(hfmm_server* server, hfmm_tree* tree, double k, int32_t P,
                       const void* b_dev, void* x_dev, double tol, int32_t restart,
                       int32_t maxit, int64_t* ticket, int64_t* footprint_bytes);
int hfmm_server_step(hfmm_server* server, void* stream, int32_t* n_active, int32_t* n_queued);
/* state: 0 queued, 1 active, 2 converged, 3 not converged (maxit), 4 stopped
 * early (hfmm_server_set_limits), -1 failed.
 * times3 (may be NULL): submit, admit and completion times (seconds, steady
 * clock). */
int hfmm_server_poll(hfmm_server* server, int64_t ticket, int32_t* state,
                     hfmm_gmres_info* info, double* times3);
/* Forgets a finished ticket. */
int hfmm_server_release(hfmm_server* server, int64_t ticket);
int hfmm_server_used_bytes(hfmm_server* server, int64_t* used);
void hfmm_server_free(hfmm_server* server);

/* Statistics of the tree and, if P > 0, of the prepared (k, P) operator. */
int hfmm_tree_stats(hfmm_tree* tree, double k, int32_t P, hfmm_stats* out);

/* Host copies of the tree for structural tests (no device access).
 *  P = 0: the base tree (split on ncrit only).  P > 0: the tree used at
 *  (k, P), where non-empty cells wider than kappa/k also split (such cells
 *  could never be accepted for M2L).
 *  src_perm/tgt_perm: int32[n_src]/[n_tgt], sorted position -> input index.
 *  cells: int32[n_cell][10] = level, i, j, k (cell coordinates at its level),
 *  src_begin, src_end, tgt_begin, tgt_end, child_begin, child_end
 *  (n_cell from hfmm_tree_stats with the same k, P).  Any pointer may be NULL. */
int hfmm_tree_export(hfmm_tree* tree, double k, int32_t P, int32_t* src_perm,
                     int32_t* tgt_perm, int32_t* cells);

/* Host copies of the traversal lists at (k, P): int32 pairs (target cell,
 * source cell), n_m2l and n_p2p of them (hfmm_tree_stats gives the counts).
 * Builds the lists on the host if needed; touches no device memory. */
int hfmm_lists_export(hfmm_tree* tree, double k, int32_t P, int32_t* m2l_pairs,
                      int32_t* p2p_pairs);

/* Per-phase device times (ms) of the last hfmm_matvec while timing is on,
 * from HIP events recorded on the call's stream around each launch group:
 * [0] P2M (with clearing and gathering the strengths), [1] M2M, [2] M2L
 * matrix-core kernel, [3] M2L reduction, [4] L2L, [5] L2P, [6] P2P, [7]
 * output scatter and BIE corrections, [8] total, [9] unused.
 * hfmm_set_timing(tree, 1) turns the events on (they add a little overhead). */
int hfmm_set_timing(hfmm_tree* tree, int32_t on);
int hfmm_phase_times(const hfmm_tree* tree, float* ms10);

/* Launch-shape autotuning of the fused matvec.  Phase 0 is the M2L
 * matrix-core kernel (shapes: pairs per wave, waves per SIMD, chunks per
 * wave, table prefetch distance); phase 1 is the P2P near-field kernel
 * (variants: waves per block x source stages per LDS tile x where the P2P
 * forks off beside the far field: right after the gather, or after the
 * M2L, beside its reduction).  The variants of a phase compute
 * bit-identical results; by default the first product of each fused
 * sequence (a tree's plain matvec, a batch, a server composition) times
 * every variant of each phase on its own work (the M2L alone, the P2P
 * inside the whole product), outside any graph capture, and keeps the
 * fastest, cached per (phase, P, log2 of the phase's work items).
 *  hfmm_variant_count: number of shapes of `phase` at order P (>= 1), or
 *    HFMM_EINVAL.
 *  hfmm_set_variant: variant >= 0 forces that shape (ignored where it does
 *    not exist for P); -1 restores tuning.  Process-wide; a captured graph
 *    is re-captured when its shape changes.
 *  hfmm_tree_variant: the shape the plain matvec of (tree, k, P) uses, or -1
 *    before its first product.
 * Phase 2 (BIE handles) is where the GMRES product adds the near
 * corrections: 0 after the FMM, 1 on a stream of the handle's own beside
 * it (the same bits); the first hfmm_gmres_solve of each (k, P) times both,
 * and hfmm_tree_variant reports the placement its next product uses (-1
 * for a (k, P) not yet prepared).
 * With the environment variable HFMM_TUNE_CACHE naming a file, the choices
 * are read from it on first use (lines "phase P log2size variant") and each
 * new choice is appended, so later processes reuse them without timing. */
int hfmm_variant_count(int32_t phase, int32_t P);
int hfmm_set_variant(int32_t phase, int32_t variant);
int hfmm_tree_variant(hfmm_tree* tree, double k, int32_t P, int32_t phase, int32_t* variant);

void hfmm_tree_free(hfmm_tree* tree);
const char* hfmm_last_error(void);
int hfmm_version(void);

/* Test hook: one M2L translation (eq. (12)-(14) translated between cells,
 * Sec. 2.3) applied to `count` expansion vectors through the product's own
 * translation-table generator, reflection codes, matrix-core M2L kernel and
 * fixed-order reduction, so the M2L can be checked coefficient by
 * coefficient.  Column c is the pair (target c, source c) whose offset,
 * target centre minus source centre, is the canonical vector t_host
 * (t0 >= t1 >= 0, t2 >= 0, not zero) under reflection refl_host[c] (bit 3:
 * swap x and y, then bits 0, 1, 2: negate x, y, z).  Coefficients are in the
 * product's scaled basis: in = M_n / s_n(rho_in), out = s_n'(rho_out) L_n',
 * with s_n(rho) = rho^n / (2n + 1)!!.
 *  in_dev, out_dev: complex64 [count][P^2] device memory (must not alias).
 *  Allocates, and waits on `stream` before returning.
 *  EINVAL: k, P as for hfmm_prepare, k_imag < 0, rho outside (0, 1], t not
 *  canonical, a reflection outside 0..15, count outside [1, 2^20], NULL. */
int hfmm_debug_m2l(int32_t P, double k, double k_imag, const double* t_host, double rho_in,
                   double rho_out, int32_t count, const int32_t* refl_host, const void* in_dev,
                   void* out_dev, void* stream);

/* Test hook for the error paths: after = n >= 0 makes the (n+1)-th next
 * device allocation of the library fail with HFMM_ENOMEM without calling
 * hipMalloc (then the hook turns itself off); -1 turns it off.
 * Process-wide.  EINVAL: after < -1. */
int hfmm_debug_fail_alloc(int64_t after);

#ifdef __cplusplus
}
#endif
#endif /* HFMM_H */
