/*
 * hddm.h -- C ABI of the MI355X (gfx950) library for the one-step overlapping
 * domain-decomposition preconditioner of Leng & Ju for the 2D Helmholtz
 * equation truncated by a uniaxial PML.
 *
 * What is computed (paper: Sec. 2 and Sec. 3):
 *   * The truncated problem J^-1 div(A grad u) + k^2 u = f (Sec. 2, eq. pml),
 *     multiplied through by J and discretised with the second-order 5-point
 *     stencil on a cell-centred grid (Sec. 3):  M u = b with b = J f = f
 *     (f vanishes outside the interior).  M is complex symmetric.
 *   * Nb_x x Nb_y non-overlapping tiles (Sec. 2); the first/last tile along an
 *     axis also takes the adjacent global PML strip, so tiles partition all
 *     nodes.  Each tile is widened by the overlap on interior sides and wrapped
 *     in its own PML (Sec. 2, the overlapping subdomains and Fig. 1).
 *   * The one-step preconditioner (Sec. 2, eq. ddm0 and eq. pc):
 *       z = sum over boxes of  E_box  M_box^-1  R~_box r,
 *     with R~ keeping r on the tile only and E adding the local solution back
 *     over the whole box, layer included.
 *   * Restarted FGMRES with this preconditioner (Sec. 3: GMRES with restart
 *     and a relative tolerance) in FP64.
 *
 * Grid conventions.  nx, ny interior nodes per axis, spacing h (the interior is
 * [0, nx h] x [0, ny h]), npml PML cells on each side, so the truncated grid has
 * Ngx = nx + 2 npml by Ngy = ny + 2 npml nodes; node g sits at (g - npml + 1/2) h.
 * Stretch a(t) = 1 + i * sigma0_over_kref * (d/L)^pml_power with d the distance
 * outside the physical interval and L = npml h.  u = 0 one node past the grid.
 *
 * Vector layout.  Every vector argument is a DEVICE pointer to Ngy*Ngx complex
 * values, row-major (y outer, x fastest), interleaved (re, im) doubles
 * ("c128").  Velocity is a HOST array of Ngy*Ngx doubles in the same order.
 *
 * Ownership.  The caller allocates and owns every device buffer (factor, work,
 * Krylov).  The library never allocates device memory; it keeps host tables
 * inside the context, and one fixed 64 MiB array per device that comes with
 * its code object (used only by hddm_apply_precond_noalloc).  Nothing is
 * freed by the library except the context.
 *
 * Errors.  Every entry point returns an hddm_status; on failure
 * hddm_last_error() returns a thread-local message.  No exception or abort
 * crosses the ABI.  State machine: setup -> bind -> factor -> apply/matvec/
 * solve; calls out of order return HDDM_ESTATE.  One context must not be used
 * from two streams at once; distinct contexts may run concurrently.
 *
 * Streams.  `stream` arguments are hipStream_t values passed as void* (NULL is
 * the default stream).  Launches are asynchronous on that stream except where
 * stated.
 */
#ifndef HDDM_H
#define HDDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hddm_ctx hddm_ctx;

typedef enum {
  HDDM_OK = 0,
  HDDM_EINVAL = 1,      /* invalid argument or layout */
  HDDM_ENOMEM = 2,      /* a caller buffer is too small */
  HDDM_ESTATE = 3,      /* call out of order (e.g. apply before factor) */
  HDDM_ENOCONV = 4,     /* solve hit maxit; info and x hold the last iterate */
  HDDM_EBREAKDOWN = 5,  /* non-finite value in the Krylov recurrence */
  HDDM_EDEVICE = 6      /* a HIP runtime call failed */
} hddm_status;

typedef enum {
  HDDM_PLAIN_C128 = 0,  /* local factors and sweeps in complex FP64 */
  HDDM_MIXED_C64 = 1    /* local factors and sweeps in complex FP32 (MFMA
                           factor); matvec, Arnoldi and least squares FP64 */
} hddm_precision;

typedef struct {
  int32_t nx, ny;            /* interior nodes per axis (multiples of tile) */
  int32_t npml;              /* PML cells per side (>= 1) */
  int32_t tile;              /* tile side n in nodes (even) */
  int32_t n_ol;              /* overlap in nodes on interior sides (even, >= 0) */
  int32_t pml_power;         /* profile exponent (2: quadratic) */
  int32_t precision;         /* hddm_precision */
  int32_t factor_format;     /* 0: automatic -- complex64 keeps only the 16x16
                                tiles on and above the diagonal of each
                                complex-symmetric G_j (half the bytes streamed
                                per sweep; boxes up to 256 wide), complex128
                                stores G_j dense; 1: dense column-major;
                                2: nested dissection -- the low-fill direct
                                local solver (Sec. 3 leaves the local solver
                                open): each box is split by separator lines
                                across the longer side of its rectangles down
                                to 16 nodes and factorised by the multifrontal
                                method, front by front G = A_ss^-1 and
                                L = -A_bs G in complex128 (about 74 entries per
                                node instead of 88 for the packed line
                                factor); precision HDDM_MIXED_C64 only (the
                                vectors are complex64).  The single-form
                                entry points run the same kernels with one
                                column, in a block workspace of 16 planes
                                reserved inside the work buffer, so a
                                single-form application streams the fronts
                                and costs about what a 16-column block
                                application costs */
  double h;                  /* grid spacing */
  double omega;              /* angular frequency; k^2 = (omega / c)^2 */
  double k_ref;              /* reference wave number of the stretch */
  double sigma0_over_kref;   /* sigma0 / k_ref (20 in the default profile) */
} hddm_problem;

typedef struct {
  double tol;        /* relative residual ||b - M x|| / ||b|| to reach */
  int32_t restart;   /* FGMRES cycle length m (<= the value given to query_bytes) */
  int32_t maxit;     /* maximum total Arnoldi steps */
  int32_t ortho;     /* Gram-Schmidt: 0 = classical, applied twice (two passes
                        of inner products and two of updates over the basis);
                        1 = the same CGS2 with the second projection's
                        coefficients taken from the Gram matrix of the basis,
                        V^H (w - V p) = p - (V^H V) p with p = V^H w (one pass
                        forms p and the new Gram column, one pass updates) */
  int32_t reserved;
} hddm_solve_opts;

typedef struct {
  int32_t iters;       /* total Arnoldi steps (= preconditioner applications) */
  int32_t restarts;    /* FGMRES cycles started */
  double relres_est;   /* last Givens residual estimate |gamma| / ||b|| */
  double relres_true;  /* ||b - M x|| / ||b|| recomputed at the end */
  int32_t status;      /* hddm_status of the solve */
  int32_t reserved;
} hddm_solve_info;

/* Build host tables for one medium: PML stretch at nodes and flux points
 * (Sec. 2, eq. pml), tile and box ranges (Sec. 2), per-box stretch tables
 * (each box's own layer, Sec. 2 eq. pmlij), descriptor and gather tables.
 * velocity: host, Ngy*Ngx doubles, positive.  Touches no GPU except to record
 * `device`.  Rejects: non-positive sizes, nx/ny not multiples of tile, odd tile
 * or n_ol, tile < 2 (n_ol + npml) when there is more than one tile (a node
 * must lie in at most two boxes per axis), non-positive velocity, unknown
 * precision.  *out receives a new context (free with hddm_destroy). */
hddm_status hddm_setup(const hddm_problem* prob, const double* velocity, int32_t device,
                       hddm_ctx** out);

/* Device bytes the caller must provide: factor_bytes for the local inverse
 * Schur complements (per box my blocks: mx^2 entries dense, or
 * 256 * nt(nt+1)/2 entries packed with nt = ceil(mx/16); c64 or c128; for
 * factor_format 2 the fronts' G, L and L^T), work_bytes for device tables,
 * the box-solution workspace and (packed format) the factor's working
 * matrices -- with factor_format 2 also the fronts' working matrices, the
 * update matrices of two tree depths and a 16-column block workspace that
 * the single-form entry points run in (about 28 GB at 4096^2, 12.6 GB of it
 * that block workspace, reserved whether or not single-form calls are made)
 * -- and krylov_bytes for one solve with FGMRES cycle length `restart`.  Any
 * output pointer may be NULL. */
hddm_status hddm_query_bytes(const hddm_ctx* ctx, int32_t restart, size_t* factor_bytes,
                             size_t* work_bytes, size_t* krylov_bytes);

/* Attach caller-owned device buffers (256-byte aligned) and upload the tables
 * (synchronous on `stream`).  Buffers must stay valid until hddm_destroy or the
 * next bind.  ENOMEM if a size is below hddm_query_bytes. */
hddm_status hddm_bind(hddm_ctx* ctx, void* factor_buf, size_t factor_bytes, void* work_buf,
                      size_t work_bytes, void* stream);

/* Factor every local problem (Sec. 3: local problems are factorised once by a
 * direct solver and reused): for each box, ordered by x-lines,
 * S_0 = T_0, S_j = T_j - B_{j-1} S_{j-1}^-1 B_{j-1}, and G_j = S_j^-1 is stored
 * in the problem's factor format (symmetric-packed upper 16x16 tiles, or
 * dense column-major).  T_j is the tridiagonal x-line block and B_j the
 * diagonal coupling of lines j and j+1.  Each S_j is inverted by blocked
 * Gauss-Jordan without pivoting; in complex64 by default on the matrix cores
 * with symmetric elimination (S_j is complex symmetric; variants in
 * hddm_tune).  With factor_format 2, the multifrontal factorisation
 * of the nested-dissection order instead, one launch per separator-tree depth
 * from the leaves.  Asynchronous. */
hddm_status hddm_factor(hddm_ctx* ctx, void* stream);

/* Pivot diagnostic of the line factor (Sec. 3: local problems factorised by
 * a direct solver; here every S_j is inverted by Gauss-Jordan without
 * pivoting).  For box b (lexicographic order), out[2 b] and out[2 b + 1]
 * receive the smallest and the largest relative pivot |p_k| / |S_j(k, k)|
 * over all lines j and positions k, as computed in the factor's own
 * precision: p_k is the k-th pivot of the unpivoted elimination of S_j (the
 * ratio of its leading principal minors of orders k+1 and k) and S_j(k, k)
 * the diagonal entry it started from.  A smallest value far below 1 flags
 * cancellation on the diagonal, i.e. a box whose unpivoted factor lost
 * accuracy; the layer-damped boxes of the benchmark and serving media give
 * 0.5 - 1 (FP64 reference in the tests).  out: host, 2 * nboxes floats.
 * Synchronises `stream` (the one hddm_factor ran on) and copies.  ESTATE
 * before hddm_factor or on a context factored through hddm_share_factor
 * (query the source), EINVAL for the nested-dissection factor
 * (factor_format 2), whose front pivots are not recorded. */
hddm_status hddm_factor_pivots(hddm_ctx* ctx, float* out, void* stream);

/* Reuse the factorisation of `src` in `dst` (factors kept resident and
 * reused across right-hand sides; Sec. 3: the local factorisation is a
 * one-time setup).  Both contexts must describe the same problem (sizes,
 * layout, precision, factor format, stretch and medium) and `dst` must be bound to the same
 * factor buffer as `src`, with its own work buffer; `src` must be factored.
 * Then `dst` is factored too, and the two contexts may run applies and solves
 * concurrently on different streams (the factor is only read).  EINVAL if the
 * problems or factor buffers differ, ESTATE if `src` is not factored or `dst`
 * is not bound.  Host only. */
hddm_status hddm_share_factor(hddm_ctx* dst, const hddm_ctx* src);

/* z = P^-1 r (Sec. 2, eq. ddm0 + eq. pc): restrict r to every tile, run the
 * block forward/backward sweeps of every box, and sum the box solutions,
 * layer included, into z in a fixed order (deterministic).  r and z are
 * c128 device vectors and must not overlap.  Asynchronous. */
hddm_status hddm_apply_precond(hddm_ctx* ctx, const void* r, void* z, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): hddm_apply_precond
 * with the box solutions between the local sweeps and the sum held in a
 * fixed array of this library (64 MiB per device, allocated when the library
 * is loaded and held until the process ends) instead of the caller's work
 * buffer; each kernel is launched directly (no graph objects are created).
 * Same kernels and order as hddm_apply_precond, so bitwise the same z.
 * Needs the line factor (factor_format 0 or 1; EINVAL for 2) and box
 * solutions of at most 64 MiB (sum over boxes of mx * my entries of 8 bytes
 * in complex64, 16 in complex128: up to 2048^2 grids with 128-node tiles in
 * complex64); EINVAL beyond, before any device work.  Every call on a device
 * shares that device's array: calls that overlap in time on one device (other
 * streams, other threads, other contexts) race and must be serialised by the
 * caller.  No part of the array needs clearing: every entry read is written
 * first in the same call.  Allocates nothing, no hipMalloc/hipFree.
 * Asynchronous. */
hddm_status hddm_apply_precond_noalloc(hddm_ctx* ctx, const void* r, void* z, void* stream);

/* y = M x, the global 5-point PML operator (Sec. 2 eq. pml times J; Sec. 3),
 * FP64.  x and y are c128 device vectors and must not overlap.  Asynchronous. */
hddm_status hddm_matvec(hddm_ctx* ctx, const void* x, void* y, void* stream);

/* Solve M x = rhs (Sec. 3: the one-step preconditioner of Sec. 2 eq. pc used
 * inside restarted GMRES to a relative tolerance) by FGMRES(restart) with
 * x0 = 0, the preconditioner applied from the right, stopping when
 * ||rhs - M x|| / ||rhs|| <= tol (estimated by the Givens recurrence, then
 * confirmed on the true residual at the end of a cycle).  Arnoldi uses classical Gram-Schmidt applied twice, in FP64 (see
 * hddm_solve_opts.ortho for the two ways of computing it).
 * krylov_buf: device scratch of hddm_query_bytes(restart) bytes.  Blocks the
 * host (one small device-to-host copy per Arnoldi step).  info may be NULL.
 * Returns HDDM_ENOCONV after maxit steps (x holds the last iterate). */
hddm_status hddm_solve(hddm_ctx* ctx, const void* rhs, void* x, const hddm_solve_opts* opts,
                       hddm_solve_info* info, void* krylov_buf, size_t krylov_bytes,
                       void* stream);

/* ---- Block form: several right-hand sides share each read of the factors.
 * The apply of Sec. 2 eq. pc is linear in r, so nrhs residuals are restricted
 * together and every step of the two sweeps becomes G_j times an mx x 16
 * panel (one GEMM on the matrix cores instead of nrhs GEMVs); the result for
 * each right-hand side equals the single form's up to complex64 rounding.
 * Needs complex64 symmetric-packed factors (precision HDDM_MIXED_C64,
 * factor_format 0) and boxes at most 192 nodes wide, or the nested-dissection
 * factor (factor_format 2: one forward launch per depth of the separator tree
 * from the leaves, then one backward launch per depth from the root); EINVAL
 * otherwise. */
#define HDDM_BLOCK_MAX 16

/* Device bytes of the block workspace (box solutions and sources of 16
 * right-hand sides, complex64, independent of nrhs) and of the Krylov buffer
 * of hddm_solve_block for nrhs right-hand sides and this restart. */
hddm_status hddm_query_block_bytes(const hddm_ctx* ctx, int32_t nrhs, int32_t restart,
                                   size_t* block_work_bytes, size_t* krylov_bytes);

/* z_k = P^-1 r_k for k < nrhs (1..16): r_k at r + k*ldr and z_k at z + k*ldz
 * (c128 device vectors, strides in complex entries, at least the grid size
 * when nrhs > 1; inputs and outputs must not overlap).  block_work: caller's
 * device buffer of hddm_query_block_bytes bytes, 256-byte aligned; its content
 * is scratch.  Deterministic.  Asynchronous. */
hddm_status hddm_apply_precond_block(hddm_ctx* ctx, const void* r, int64_t ldr, void* z,
                                     int64_t ldz, int32_t nrhs, void* block_work,
                                     size_t block_work_bytes, void* stream);

/* hddm_solve for nrhs (1..16) right-hand sides at once: each runs its own
 * FGMRES (same options, own Krylov region) and every preconditioner
 * application serves all of them still iterating, through the block form.
 * rhs_k at rhs + k*ldb, x_k at xout + k*ldx (c128 device vectors).
 * info: array of nrhs entries (may be NULL).  krylov_buf: device buffer of
 * hddm_query_block_bytes(nrhs, restart) bytes.  Returns the worst status
 * (EBREAKDOWN before ENOCONV before OK); per-RHS status in info.  Blocks the
 * host: one small copy per round for all right-hand sides. */
hddm_status hddm_solve_block(hddm_ctx* ctx, const void* rhs, int64_t ldb, void* xout,
                             int64_t ldx, int32_t nrhs, const hddm_solve_opts* opts,
                             hddm_solve_info* info, void* block_work, size_t block_work_bytes,
                             void* krylov_buf, size_t krylov_bytes, void* stream);

/* Convergence history of the last completed solve on ctx (hddm_solve,
 * hddm_solve_block, or a session problem once hddm_session_result has
 * returned it): the residual estimate |gamma_{j+1}| / ||b|| of the Givens
 * recursion of restarted GMRES (Sec. 3) after every Arnoldi step, in step
 * order across the restarts (each cycle starts again from the true residual
 * of the previous one).  rhs: right-hand side index of that solve (0 for
 * hddm_solve).  out: host array of cap doubles (may be NULL when cap is 0);
 * min(cap, steps) values are copied and *n receives the number of steps
 * (equal to the solve's info.iters).  EINVAL for a null context or n, an rhs
 * outside the last solve or a negative cap; ESTATE if no solve has completed
 * on ctx.  Host only, no GPU work. */
hddm_status hddm_solve_history(const hddm_ctx* ctx, int32_t rhs, double* out, int32_t cap,
                               int32_t* n);

/* ---- Several problems in one launch (serving): the preconditioner of
 * Sec. 2 eq. pc applied for n contexts at once -- n restrictions, ONE block
 * sweep launch over the union of all their boxes (each box with its own
 * factor, stretch tables, sources and solutions), n sums -- so problems of
 * different grids, media and wave numbers share the device in one launch
 * sequence (a graph launch while hddm_use_graphs is on for ctxs[0], whose
 * graph cache and event timing it uses).  Every context must be factored
 * with the block form of the line factor (complex64 symmetric-packed, boxes
 * at most 192 wide), all with boxes of the same tile-block width (e.g. tiles
 * of 128 with overlap 8 and a 16-cell layer, at any grid size) on one
 * device, each at most once; n in 1..HDDM_BATCH_MAX.  The batch's results
 * equal each context's own hddm_apply_precond_block bitwise. */
#define HDDM_BATCH_MAX 8

/* For i < n: z_i,k = P_i^-1 r_i,k for k < nrhs[i] (1..16), r_i,k at
 * r[i] + k*ldr[i], z_i,k at z[i] + k*ldz[i] (c128 device vectors of context
 * i's grid), block_work[i]: context i's block workspace (as for
 * hddm_apply_precond_block).  EINVAL / ENOMEM / ESTATE as there.
 * Asynchronous. */
hddm_status hddm_apply_precond_batch(hddm_ctx* const* ctxs, int32_t n, const void* const* r,
                                     const int64_t* ldr, void* const* z, const int64_t* ldz,
                                     const int32_t* nrhs, void* const* block_work,
                                     const size_t* block_work_bytes, void* stream);

/* A solver session: block FGMRES problems (hddm_solve_block's, Sec. 3) of up
 * to HDDM_BATCH_MAX contexts advanced together, one round per
 * hddm_session_step: every round applies the preconditioner for all their
 * iterating right-hand sides in one fused launch sequence (as
 * hddm_apply_precond_batch), then runs each problem's Arnoldi steps, reads
 * all summaries with one wait and updates the Givens rotations.  Problems
 * may be added between steps while others iterate (continuous batching) and
 * leave when they finish.  A problem's iterates, counts and results are
 * bitwise those of hddm_solve_block on its own (the same kernels per box and
 * per right-hand side, in the same order).  Contexts as for
 * hddm_apply_precond_batch; a context may hold one problem at a time and
 * must not be used elsewhere while it does; all steps on one stream.  Host
 * objects only: the caller owns every device buffer. */
typedef struct hddm_session hddm_session;
hddm_status hddm_session_create(hddm_session** out);

/* Adds the solve of ctx's nrhs (1..16) right-hand sides rhs + k*ldb into
 * xout + k*ldx (c128 device vectors), options, block workspace and Krylov
 * buffer as for hddm_solve_block (the buffers stay in use until the problem
 * is collected by hddm_session_result).  *id receives the problem's handle.
 * Nothing runs until the next hddm_session_step.  EINVAL if the session holds
 * HDDM_BATCH_MAX problems, ctx already has one, or its boxes differ in
 * tile-block width from the others'. */
hddm_status hddm_session_add(hddm_session* s, hddm_ctx* ctx, const void* rhs, int64_t ldb,
                             void* xout, int64_t ldx, int32_t nrhs, const hddm_solve_opts* opts,
                             void* block_work, size_t block_work_bytes, void* krylov_buf,
                             size_t krylov_bytes, int32_t* id);

/* One round of every problem of the session (problems added since the last
 * step start with x = 0 and their first residual).  Blocks the host: two
 * waits per round at most.  finished: caller array of HDDM_BATCH_MAX entries
 * receiving the ids of the problems that finished in this step (all their
 * right-hand sides converged, reached maxit or broke down), *nfinished their
 * number. */
hddm_status hddm_session_step(hddm_session* s, void* stream, int32_t* finished,
                              int32_t* nfinished);

/* A finished problem's per-RHS info (nrhs entries; may be NULL) and status
 * (the worst of its right-hand sides, as hddm_solve_block), and its removal
 * from the session.  ESTATE if it is still iterating, EINVAL for an unknown
 * id. */
hddm_status hddm_session_result(hddm_session* s, int32_t id, hddm_solve_info* info);

/* Frees the session's host objects (problems still in it are dropped). */
hddm_status hddm_session_destroy(hddm_session* s);

/* Block-form kernel choice (any time after setup; takes effect on the next
 * launch): 0 = automatic (as 1), 1 = three real MFMAs per complex product
 * (P1 = Re U Re V, P2 = Im U Im V, P3 = (Re U + Im U)(Re V + Im V),
 * Re = P1 - P2, Im = P3 - P1 - P2: a quarter fewer matrix-core operations,
 * complex64 rounding of the imaginary part up to about twice that of the
 * four-product form) with each tile's transpose formed in LDS, 2 = four real
 * MFMAs with the transpose read from memory, 3 = three real MFMAs with the
 * transpose read from memory.  EINVAL on other values. */
hddm_status hddm_tune_block(hddm_ctx* ctx, int32_t variant);

/* Graph replay of the preconditioner application (Sec. 2 eq. pc: restrict,
 * all local solves, sum).  enable != 0 (the default): the launches of one
 * application go to the device as one hipGraph launch: in the block form the
 * restriction of a stand-alone application, the sweep over all boxes and the
 * gather; in the single form the sweep (restricting r itself) and the gather.
 * The graph is built once per kernel choice and launch shape, kept in the
 * context and replayed with each call's arguments, including inside the
 * block solve.  enable == 0: the same kernels are launched one by one.  The
 * results are bitwise identical either way.  EINVAL for a null context. */
hddm_status hddm_use_graphs(hddm_ctx* ctx, int32_t enable);

/* Smoothing function of the Remark after eq. pc (Sec. 2): enable != 0
 * multiplies each local solution by its box's beta_ij before the sum, in
 * every application (single and block form, stand-alone and inside the
 * solves); 0 (the default) is the plain sum of the paper's experiments.  The
 * paper asks only that beta be C^2, 1 on the tile and 0 outside the box;
 * here beta_ij(x, y) = b_i(x) b_j(y) with b = 1 on the tile and, across each
 * interior side's strip of L nodes (overlap and local layer), b = 1 - S(s) at
 * s = (d + 1/2) / L for the node d nodes past the tile edge, S(s) = 10 s^3 -
 * 15 s^4 + 6 s^5 (global-boundary sides have no strip).  Takes effect on the
 * next application; EINVAL for a null context. */
hddm_status hddm_set_smoothing(hddm_ctx* ctx, int32_t enable);

/* The iterative multi-step DDM as a solver (Sec. 2, eq. ddm0, eq. ddms and
 * eq. sum): step 0 solves every box with the right-hand side on its tile;
 * step s+1 solves every box with minus the sum of its neighbours' residuals
 * (the operator applied to their step-s local solutions) on its tile; x is
 * the sum of all local solutions of all steps.  Because a local solution
 * leaves no residual on its own tile, the step-(s+1) sources over all tiles
 * are r_{s+1} = r_s - M z_s (z_s: the sum of step s's local solutions, r_0 =
 * b), which is how they are formed here: every step is one preconditioner
 * application (graph launch), x += z_s and one stencil product.
 * rhs, xout: device c128 vectors of the global grid (xout overwritten); stops
 * after max_steps (>= 1) steps or once |r_s| / |b| <= tol (>= 0).  info
 * (optional): iters = steps taken, restarts = 0, relres_est = |r_s| / |b|,
 * relres_true = |b - M x| / |b| recomputed at the end, status.  work: device,
 * 256-byte aligned, at least hddm_ddm_query_bytes bytes.  Returns ENOCONV if
 * max_steps is reached first, EBREAKDOWN on a non-finite residual, ESTATE
 * before hddm_factor. */
hddm_status hddm_ddm_query_bytes(const hddm_ctx* ctx, size_t* work_bytes);
hddm_status hddm_ddm_solve(hddm_ctx* ctx, const void* rhs, void* xout, int32_t max_steps,
                           double tol, hddm_solve_info* info, void* work, size_t work_bytes,
                           void* stream);

/* Release the context and its host tables (device buffers stay the caller's). */
hddm_status hddm_destroy(hddm_ctx* ctx);

/* Thread-local message of the last failing call ("" if none). */
const char* hddm_last_error(void);

/* Geometry introspection (host only).  Writes nbx, nby and, if `boxes` is not
 * NULL, 8 int32 per box in lexicographic order (y outer, x inner): box x range
 * [x0, x1), box y range [y0, y1), tile x range, tile y range, all in global
 * node indices, half-open. */
hddm_status hddm_geometry(const hddm_ctx* ctx, int32_t* nbx, int32_t* nby, int32_t* boxes);

/* Host copies of the global stretch tables (for tests): a_x at Ngx nodes and
 * Ngx+1 flux points, then a_y likewise, as interleaved complex doubles; out
 * must hold 2*(2 Ngx + 1 + 2 Ngy + 1) doubles. */
hddm_status hddm_stretch_tables(const hddm_ctx* ctx, double* out);

/* Kernel selection (for the autotuner; any call order after setup, takes
 * effect on the next launch).  sweep_variant, dense complex64 format: 0 =
 * automatic (wave-structured sweep when the boxes fit one per CU, otherwise
 * one row per thread), 1 = wave-structured, 2 = one row per thread;
 * symmetric-packed format: 0 = one workgroup per CU with no register cap,
 * 1 = register cap for two workgroups (boxes) per CU, 2 = as 0.  sweep_threads: threads
 * per workgroup of the one-row-per-thread sweep (0 = automatic; rounded up to
 * a multiple of 64, at least the widest box, at most 1024).  factor_variant
 * (complex64; each inverse G_j = S_j^-1 by blocked Gauss-Jordan with 16-wide
 * blocks on the matrix cores unless stated): 0 = automatic (4 for boxes up to
 * 192 wide, else 2), 1 = vector FMA, 2 = working matrix in memory, 3 = working
 * matrix in registers (the same arithmetic as 2 in the same order: bitwise
 * equal factors), 4 = symmetric elimination in registers (S_j is complex
 * symmetric: only the tiles on and above the diagonal are updated, half the
 * work of 3; the same pivots, factors equal to 3 up to FP32 rounding).
 * complex128 always uses the one-row-per-thread sweep and the vector factor.
 * EINVAL on other values. */
hddm_status hddm_tune(hddm_ctx* ctx, int32_t sweep_variant, int32_t sweep_threads,
                      int32_t factor_variant);

/* Kernel timing with HIP events (for benchmarks).  While enabled, every launch
 * made through `ctx` is bracketed by a pair of events recorded on the launch
 * stream and its duration is accumulated per kernel class:
 *   HDDM_K_SWEEP (restriction + forward/backward sweeps of all boxes; block
 *   form: the sweeps only), HDDM_K_GATHER (sum of the box solutions),
 *   HDDM_K_MATVEC, HDDM_K_KRYLOV (Gram-Schmidt, norms, scaling, solution
 *   update, true residual), HDDM_K_FACTOR, HDDM_K_RESTRICT (block form's
 *   restriction).
 * Enabling/disabling resets the counters.  hddm_profile_read synchronises the
 * stream of the last launch, then reports launches and total milliseconds. */
enum { HDDM_K_SWEEP = 0, HDDM_K_GATHER = 1, HDDM_K_MATVEC = 2, HDDM_K_KRYLOV = 3,
       HDDM_K_FACTOR = 4, HDDM_K_RESTRICT = 5, HDDM_K_COUNT = 6 };
hddm_status hddm_profile(hddm_ctx* ctx, int32_t enable);
hddm_status hddm_profile_read(hddm_ctx* ctx, int32_t kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* HDDM_H */
