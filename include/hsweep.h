/*
 * hsweep -- moving-PML sweeping preconditioner for the 7-point heterogeneous
 * 3D Helmholtz operator on one MI355X (gfx950).
 *
 * The problem is the one of Poulson, Engquist, Li and Ying, "A parallel
 * sweeping preconditioner for heterogeneous 3D Helmholtz equations":
 * given the velocity c(x), the angular frequency omega and a grid, solve
 * A u = f with A = -Delta - omega^2/c^2 (Sec. 1, Eq. 1.1) discretised by
 * second-order finite differences with PML, using GMRES(k) (Sec. 2.4)
 * preconditioned by the sweep (Sec. 1.1, Algs. 1.3-1.5) over panels whose
 * auxiliary problems H_i are factored by a multifrontal LDL^T over a
 * nested-dissection tree (Secs. 2.1-2.2).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Grid.  Interior nodes i_j = 1..n_j at x_j = i_j h; gamma PML nodes are
 *   added past every face, so a vector lives on the padded grid of
 *   N_j = n_j + 2 gamma nodes per axis, lexicographic with x1 fastest
 *   (index a1 + a2 N1 + a3 N1 N2), homogeneous Dirichlet just outside.
 * - Vectors are complex128 (hsw_c128, interleaved re/im).  A block of nrhs
 *   vectors stores each vector contiguously, vector r starting at r * ld,
 *   ld >= N_pad = N1 N2 N3.
 * - Pointers named as device pointers must be device memory of the device
 *   the context was created on; they are read/written in order on the
 *   context's stream.  The library keeps no caller pointer after a call
 *   returns; it owns the plan, factors and workspace until hsw_destroy.
 * - Every call returns a status and never aborts; hsw_last_error gives the
 *   message of the last failure.  A context is not thread-safe.
 */
#ifndef HSWEEP_H
#define HSWEEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsw_ctx hsw_ctx;

typedef struct {
    double re, im;
} hsw_c128;

typedef enum {
    HSW_OK = 0,
    HSW_E_INVAL = 1,     /* bad argument (size, pointer, non-positive or non-finite c) */
    HSW_E_NOMEM = 2,     /* plan does not fit in device memory; nothing allocated */
    HSW_E_STATE = 3,     /* call out of order (e.g. apply before setup) */
    HSW_E_BREAKDOWN = 4, /* zero or non-finite pivot in the unpivoted LDL^T */
    HSW_E_NOCONV = 5,    /* GMRES reached maxit; x holds the last iterate */
    HSW_E_DEVICE = 6     /* HIP runtime error */
} hsw_status;

typedef enum {
    HSW_C128 = 0,        /* fronts, sweep and GMRES in complex FP64 */
    HSW_C64 = 1,         /* fronts and sweep in complex FP32, GMRES in FP64 */
    HSW_C64_BF16GEMM = 2 /* as HSW_C64, the Schur-update GEMMs with complex BF16 inputs on the
                            BF16 matrix cores, FP32 accumulation (option "bf16_mfma") */
} hsw_precision;

/* One problem: the grid, frequency and preconditioner parameters. */
typedef struct {
    int32_t n[3];        /* interior nodes per axis */
    double h;            /* grid spacing, same on every axis */
    double omega;        /* angular frequency (Sec. 1, Eq. 1.1) */
    double alpha;        /* damping of J = -Delta - (omega + i alpha)^2/c^2 (Sec. 1.1, Eq. 1.5);
                            0 makes J = A */
    int32_t gamma;       /* PML nodes per face, physical and artificial (Sec. 1.1) */
    double pml_amp;      /* PML amplitude C in sigma(t) = (C/eta)(t/eta)^2, eta = (gamma+1) h */
    int32_t panel_depth; /* interior x3 planes per panel, d (Sec. 1.1, before Alg. 1.4) */
    int32_t leaf;        /* nested-dissection leaf lateral extent (>= 2), or 0 for the
                            default 4, the fastest leaf measured (Sec. 2.1) */
} hsw_problem;

typedef struct {
    int32_t restart_k;   /* GMRES restart length k (Sec. 2.4) */
    int32_t maxit;       /* cap on preconditioner applications per right-hand side */
    double rtol;         /* stop when ||b - A x|| / ||b|| < rtol (true residual, FP64) */
} hsw_solve_opts;

typedef struct {
    int32_t iters_max;   /* max over right-hand sides of the iteration count */
    int32_t* iters;      /* host array, sum(nrhs) entries, or NULL */
    double* relres;      /* host array, sum(nrhs) entries: final true relative residual, or NULL */
    double t_setup;      /* seconds of the last hsw_setup (device events) */
    double t_solve;      /* seconds of this hsw_solve (device events) */
    int32_t bad_problem, bad_panel, bad_front, bad_pivot; /* breakdown location, else -1 */
} hsw_solve_info;

/*
 * Plan the symbolic structure of nprob problems and allocate the factors and
 * workspace.  Builds the panels of every problem (Sec. 1.1, Alg. 1.4:
 * m = ceil(n3 / d); panel 0 also owns the bottom gamma PML planes, panel m-1
 * the top ones), the nested dissection of every panel (Sec. 2.1: full-depth
 * separators, postorder), the update sets and extend-add maps, and the level
 * schedule that batches every front of one tree depth over all panels and
 * problems into one launch.  `stream` is a hipStream_t (NULL: the default
 * stream).  Returns HSW_E_NOMEM, allocating nothing, when the factors and
 * workspace do not fit the device.  On success *out owns everything.
 */
hsw_status hsw_create(const hsw_problem* p, int32_t nprob, hsw_precision prec,
                      void* stream, hsw_ctx** out);

/*
 * Load the velocity of every problem: c[k] is a device pointer to
 * n[0]*n[1]*n[2] doubles of problem k, x1 fastest.  The values are copied;
 * c must be positive and finite (HSW_E_INVAL otherwise).  The PML stretch
 * tables are formed here; the matrix entries of A and of every H_i are
 * generated from them on the device when needed.
 */
hsw_status hsw_assemble(hsw_ctx* ctx, const double* const* c);

/*
 * Factor every auxiliary problem of every panel (Sec. 1.1, Alg. 1.4) by the
 * multifrontal partial LDL^T of Sec. 2.2, level by level over all panels and
 * problems, then form the selectively inverted fronts used by the solves.
 * Returns HSW_E_BREAKDOWN (location in hsw_solve_info of the next solve and
 * in hsw_last_error) on a zero or non-finite pivot.
 */
hsw_status hsw_setup(hsw_ctx* ctx);

/*
 * z = M^{-1} r: one application of the sweep (Sec. 1.1, Alg. 1.5) of problem
 * `prob` to nrhs vectors.  r and z are device pointers (may not alias), each
 * nrhs vectors of the padded grid with leading dimension ld.
 */
hsw_status hsw_apply(hsw_ctx* ctx, int32_t prob, const hsw_c128* r, hsw_c128* z,
                     int32_t nrhs, int64_t ld);

/*
 * hsw_apply without allocating: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops).  Same
 * arguments and result as hsw_apply, except:
 *   - nrhs is at most 15 (the single-right-hand-side passes), and the
 *     panel-solve workspace, (max auxiliary size + max update size + max
 *     child-slot size) x nrhs complex entries of the working precision,
 *     must fit the library's 128 MiB device scratch: HSW_E_INVAL otherwise,
 *     with the sizes in hsw_last_error;
 *   - the workspace is a static device array that every call on a device
 *     shares (each device holds its own copy from its first use until the
 *     process ends): calls that overlap on one device race, so serialize
 *     them (one stream, or events between streams);
 *   - the solve block shapes are those already tuned by earlier
 *     hsw_apply / hsw_solve calls, or the fixed rule: this call times
 *     nothing and captures no graph;
 *   - the context's device must be the current device (HSW_E_INVAL).
 * It calls no hipMalloc / hipFree.  Nothing in the scratch needs to start at
 * zero: every entry a pass reads was written earlier in the same call, or is
 * masked by the extend-add maps.
 */
hsw_status hsw_apply_noalloc(hsw_ctx* ctx, int32_t prob, const hsw_c128* r, hsw_c128* z,
                             int32_t nrhs, int64_t ld);

/*
 * y = T_i v: the approximate inverse Schur complement of panel i alone
 * (Sec. 1.1, Alg. 1.3: zero-extend over the artificial PML, solve with H_i,
 * extract).  v and y are device pointers to nrhs panel vectors (the panel's
 * planes [lo, hi) of the padded grid, x1 fastest), leading dimension ld
 * >= (hi - lo) N1 N2.  hsw_query keys "panel_lo"/"panel_hi" (with the panel
 * index in the key's value argument) give lo and hi.
 */
hsw_status hsw_panel_solve(hsw_ctx* ctx, int32_t prob, int32_t panel, const hsw_c128* v,
                           hsw_c128* y, int32_t nrhs, int64_t ld);

/*
 * y = A x with the undamped 7-point operator of problem `prob` (Sec. 1,
 * Eq. 1.1 with the PML stretch).  Device pointers, nrhs vectors, ld.
 */
hsw_status hsw_matvec(hsw_ctx* ctx, int32_t prob, const hsw_c128* x, hsw_c128* y,
                      int32_t nrhs, int64_t ld);

/*
 * Solve A x = b for every problem by right-preconditioned flexible GMRES(k)
 * in FP64 (Sec. 2.4) from a zero initial guess, all right-hand sides of a
 * problem advanced together.  b[k], x[k]: device pointers to nrhs[k] padded
 * vectors of problem k (ld = N_pad).  info (may be NULL) receives the
 * iteration counts and true FP64 relative residuals.
 */
hsw_status hsw_solve(hsw_ctx* ctx, const hsw_c128* const* b, hsw_c128* const* x,
                     const int32_t* nrhs, const hsw_solve_opts* opts, hsw_solve_info* info);

/*
 * Integer facts about problem `prob`.  Keys: "N_pad", "N_int", "m" (panels),
 * "N1", "N2", "N3", "fronts" (per panel), "levels", "factor_bytes",
 * "setup_flops" (the partial factorisations and the formed columns of the
 * inversion), "factor_flops", "apply_flops" (per right-hand side: one
 * multiply-add per entry of G each pass reads, see "full_inverse"),
 * "panel_lo", "panel_hi", "panel_nz", "panel_artificial" (for these four
 * *val holds the panel index on entry).
 */
hsw_status hsw_query(const hsw_ctx* ctx, int32_t prob, const char* key, int64_t* val);

/*
 * Elimination order of panel `panel`: perm_host[e] (host array of the
 * panel's auxiliary size) is the index a1 + a2 N1 + q N1 N2 of the e-th
 * eliminated node of its auxiliary box, q = 0 being the first artificial
 * plane (or the panel's first plane when it has none).
 */
hsw_status hsw_get_perm(const hsw_ctx* ctx, int32_t prob, int32_t panel, int32_t* perm_host);

/*
 * Structure of front `front` (postorder number) of a panel:
 * info[0..4] = {first elimination position, s, u, parent front (-1 root),
 * depth}; urows (may be NULL) receives the u elimination positions of the
 * update set, ascending.
 */
hsw_status hsw_get_front_info(const hsw_ctx* ctx, int32_t prob, int32_t panel, int32_t front,
                              int32_t* info, int32_t* urows);

/*
 * Host copies (upcast to complex128) of the factored front (Sec. 2.2):
 * D (s), L_TL (s x s, column-major, unit lower; the upper part is zeroed)
 * and the final coupling F_BL = F_BL^ L_F^{-T} D_F^{-1} (u x s, column-major).
 * Any output may be NULL.  Requires hsw_setup with the factors kept (option
 * keep_factors, on by default when memory allows; otherwise the factor
 * block holds the selective inverse and this returns HSW_E_STATE).
 */
hsw_status hsw_get_front(const hsw_ctx* ctx, int32_t prob, int32_t panel, int32_t front,
                         hsw_c128* D, hsw_c128* L_TL, hsw_c128* F_BL, int32_t* s, int32_t* u);

/*
 * Host copy of the selectively inverted front used by the solves (Sec. 2.2):
 * G = [L_F^{-1}; F_BL L_F^{-1}], (s+u) x s column-major, upcast to complex128.
 * Columns the inversion did not form (before g0, see the option
 * "full_inverse") are returned as zeros.
 */
hsw_status hsw_get_front_inverse(const hsw_ctx* ctx, int32_t prob, int32_t panel, int32_t front,
                                 hsw_c128* G);

/*
 * Measurement aid (not part of the method).  enable != 0 starts timing the
 * named kernel class -- "fwd" / "bwd" (the two passes of the panel solves),
 * "diag", "panel", "trailing" (Schur updates inside the pivot columns),
 * "schur" (the update of F_BR), "assemble", "inverse" (setup) or "matvec" --
 * and resets the totals: every later launch of that class on the context's
 * stream is bracketed by a pair of HIP events, and the algorithmic bytes
 * (factor blocks and vectors the launch must move, from the plan) and flops
 * of the launch are added up.  enable == 0 stops timing, synchronizes the
 * stream and returns the number of launches, the summed event-measured
 * durations in seconds and the summed bytes and flops (any output may be NULL).
 */
hsw_status hsw_kernel_timing(hsw_ctx* ctx, const char* kernel, int32_t enable, int64_t* launches,
                             double* seconds, double* bytes, double* flops);

/*
 * Options of a context.  All but "block_gmres" are execution options (not
 * part of the method; results do not depend on them beyond rounding order,
 * and the sweep is deterministic):
 *   "graph"    1: hsw_apply and hsw_solve replay the sweep of Alg. 1.5 as
 *              a HIP graph captured at the first application for a (problem,
 *              right-hand-side count), on a context-owned copy of the vector;
 *              0 (default): launch its kernels one by one on the stream.
 *   "gmres_device_test" 1: hsw_solve (GMRES(k) per right-hand side) tests
 *              convergence on the device: after every Arnoldi step a kernel
 *              counts the step and retires the right-hand sides whose
 *              residual estimate fell below rtol, and once none is left a
 *              device flag stops every later kernel of the cycle at its
 *              first instruction.  The host issues the k steps of a cycle
 *              without waiting and reads the counts back once per cycle,
 *              with the residual norms.  With "graph" 1 as well, the k steps
 *              are captured once per (problem, right-hand-side count, k) and
 *              each cycle replays them (the context's own lane only).  The
 *              iterates equal those of the default mode bit for bit; the
 *              steps issued after convergence cost their launches.  0
 *              (default): the host reads the estimates after every step.
 *   "autotune" 1 (default): at the first application for a right-hand-side
 *              group (1, 2, 3-4, 5+), time every block shape of the solve
 *              kernels per panel class and tree depth and keep the fastest;
 *              0: a fixed rule (also set by the environment variable
 *              HSW_AUTOTUNE=0 at create time).
 *   "update_order" order of the Schur-complement updates in hsw_setup:
 *              0 right-looking (each pivot block updates everything after
 *              it); 1 left-looking (each block column receives all earlier
 *              pivots before it is factored, F_BR once at the end); 2 or -1
 *              (default) hybrid: right-looking over the pivot columns, F_BR
 *              once at the end.  The factors agree to rounding.
 *   "mm_min_rhs" 1..16 (default 4): solves (hsw_solve, hsw_apply,
 *              hsw_panel_solve) with at least this many right-hand sides take
 *              the matrix-core passes, in groups of 16 (the last one padded
 *              with zeros); fewer take the single-vector passes.
 *              hsw_apply_noalloc always takes the single-vector passes.
 *   "mm_fwd_form", "mm_bwd_form" the form of the matrix-core passes (see
 *              mm_min_rhs) at every tree depth; -1 (default): the
 *              autotuner's choice per panel class and depth.  Forward
 *              (-1..7): 0 / 3 workgroups of 64 rows whose 4 / 8 waves split
 *              the contraction, 1 / 4 / 7 workgroups of 16 rows with 4 / 8 /
 *              2 waves, 2 row-split workgroups of 64 rows
 *              with the front vector staged in LDS (depths whose largest
 *              front needs more than 64 KB of it take form 0), 5 workgroups
 *              of 64 rows with the contraction split over several workgroups
 *              and a second launch summing the parts, 6 the same for items
 *              of 16 rows.  Backward (-1..8): 0
 *              workgroups of 64 columns, 1 / 2 / 3 / 8 of 16 columns with 4 /
 *              8 / 16 (complex128: 8) / 2 waves, 4 as forward 5 for columns, 5 / 6
 *              as 1 / 2 with four chunks in flight per wave, 7 as 4 for
 *              items of 16 columns.  Out of range:
 *              HSW_E_INVAL.
 *   "solve_lanes" 1..16 (default 4): hsw_solve spreads the problems of a
 *              context over this many lanes -- streams with their own
 *              workspaces, one host thread each -- so that the launch-latency
 *              bound sweeps of small problems overlap (the device runs 4
 *              hardware queues per process).  The solve kernels' block shapes
 *              are tuned on the context's stream first; the lanes' work is
 *              ordered after earlier work on the context's stream and later
 *              work after it.  With fixed block shapes (autotune 0) the
 *              results do not depend on the lane count.  One lane while a
 *              kernel class is being timed.
 *   "block_gmres" 1: hsw_solve runs block GMRES(k) (Sec. 2.4 names block
 *              variants of GMRES as a way to lower the iteration count): the
 *              right-hand sides of a problem, in groups of at most 16, share
 *              one block Krylov space; each iteration applies the sweep to
 *              the group's still unconverged columns at once, and a column
 *              leaves the block at a restart once its true relative residual
 *              is below rtol.  iters[r] counts the iterations column r took
 *              part in.  A group whose residual block is rank deficient
 *              (dependent right-hand sides) is solved by GMRES(k) per column.
 *              0 (default): GMRES(k) per right-hand side.
 *   "keep_factors" 1: hsw_setup keeps the factors L_F, D, F_BL (readable
 *              by hsw_get_front) and writes the selective inverse G to a
 *              block of its own (allocated when the option is set;
 *              HSW_E_NOMEM if it does not fit); 0: G overwrites the factor
 *              block in place (the rows of L_F^{-1} pass through a scratch and
 *              are copied over L_F), which nearly halves the factor memory,
 *              and hsw_get_front returns HSW_E_STATE.  hsw_create picks 1
 *              when the separate block fits in device memory, else 0.
 *   "inverse_by_depth" (in place only) 1: the inversion runs one tree depth
 *              at a time through a scratch of the largest depth's L_F^{-1}
 *              blocks; 0: all fronts in one launch through a scratch for
 *              every L_F^{-1} (faster: the long rows of the top fronts overlap
 *              the rest).  hsw_create picks 0 when that scratch fits, else 1.
 *   "full_inverse" 1: every column of every G is formed; 0 (default): a
 *              leaf front (one without children) of a panel with ga > 0
 *              auxiliary planes skips the columns of those planes, which no
 *              solve reads: its pivots are ordered plane by plane, the solves'
 *              vectors are zero there and the backward pass extracts only the
 *              panel's own planes.  Its first formed column is
 *              g0 = 64 floor(min(ga cells, s) / 64), cells being the front's
 *              pivots per plane (s / panel_nz); the formed columns hold the
 *              same values either way.
 *   "triangular_solves" the solve passes of a tree depth may instead run
 *              as triangular solves with the kept factors, the path selective
 *              inversion replaces (Sec. 2.2): by 64-pivot blocks, one
 *              workgroup per front, with the stored inverses of the diagonal
 *              blocks.  2 (default): the autotuner times them against the
 *              inverse passes at every depth and keeps the faster; 1: at
 *              every depth; 0: never.  They need the factors (keep_factors
 *              1); without them every depth runs the inverse passes.
 *   "bf16_mfma" (HSW_C64_BF16GEMM) 1 (default): the Schur-update GEMMs take
 *              complex BF16 inputs (rounded to nearest even) on the BF16
 *              matrix cores with FP32 accumulation; 0: the same rounded inputs
 *              multiplied on the FP32 matrix cores (products of bf16 values
 *              are exact in FP32, so the two agree to FP32 rounding of the
 *              sums).
 * Changing "keep_factors", "inverse_by_depth", "full_inverse" or "bf16_mfma"
 * requires a new hsw_setup.
 * Returns HSW_E_INVAL for an unknown key or value.
 */
hsw_status hsw_set_option(hsw_ctx* ctx, const char* key, int64_t value);

/* Message of the last failing call on ctx (or of the last failed create when ctx is NULL). */
const char* hsw_last_error(const hsw_ctx* ctx);

/* Free everything the context owns.  NULL is accepted. */
void hsw_destroy(hsw_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HSWEEP_H */
