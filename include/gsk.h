/*
 * gsk: geometric scaling GS(p) followed by restarted GMRES(m) or Bi-CGSTAB, on one
 * AMD Instinct MI355X (gfx950). C ABI.
 *
 * Paper: D. Gordon, R. Gordon, "Geometric scaling: a simple preconditioner for certain
 * linear systems with discontinuous coefficients" (2009). The problem statement is in
 * section 2: a consistent system A x = b (eq. (1)) with no zero row; D = diag(1/||a_i||_p);
 * the geometrically scaled system D A x = D b (eq. (2)); Krylov solution from x0 (section
 * 2.1) with the relative-residual stopping test of section 2.2.
 *
 * Conventions for every entry point:
 *  - Matrix, vector and workspace pointers are DEVICE pointers (HIP device memory of the
 *    current device), owned by the caller. The library never frees them and keeps no
 *    pointer after the call returns. Vectors are dense FP64 arrays of length n.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). All device work
 *    is enqueued on it. Entry points that report results to the host (gs_scale's error
 *    checks, the solvers' gsk_info, arnoldi's step count) synchronise that stream before
 *    returning; gsk_spmv does not.
 *  - The return value is GSK_OK (0) or a negative GSK_ERR_* code; gsk_last_error() then
 *    gives a message (thread-local, valid until the next call from the same thread).
 *    Non-convergence of a solver is not an error: it is reported in gsk_info.status.
 *  - CSR matrices have int32 row pointers and column indices (0-based, columns sorted
 *    ascending within each row, no duplicates) and FP64 values. The solvers and gsk_spmv also
 *    take structured stencil matrices (gsk_matrix, gsk_stencil).
 *  - Nothing is thrown across the ABI.
 */
#ifndef GSK_H
#define GSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSK_VERSION 3

/* Return codes */
#define GSK_OK 0
#define GSK_ERR_INVALID_ARG (-1) /* bad size, NULL pointer, p < 1, m out of range, ...     */
#define GSK_ERR_ZERO_ROW (-2)    /* a row of A is zero: the paper's assumption is violated */
#define GSK_ERR_NONFINITE (-3)   /* NaN or Inf in A or b, or a row norm overflowed          */
#define GSK_ERR_WORKSPACE (-4)   /* workspace NULL, too small or misaligned (256 B)         */
#define GSK_ERR_DEVICE (-5)      /* a HIP runtime call failed                               */

/* Solver outcomes (gsk_info.status) */
#define GSK_CONVERGED 0  /* true relative residual below tol                               */
#define GSK_MAXIT 1      /* iteration cap reached (the paper's cap is 10,000, section 2.2)  */
#define GSK_BREAKDOWN 2  /* a Krylov breakdown test fired (see gsk_options.breakdown_eps)  */
#define GSK_STAGNATED 3  /* three recursive estimates below tol in a row failed the true    */
                         /* residual check (the updated residual drifted from b - A x)      */

/* Breakdown tests (gsk_info.breakdown_test) */
#define GSK_BRK_NONE 0
#define GSK_BRK_SIGMA 1   /* Bi-CGSTAB: |(r^, A p)| <= eps_b ||r^|| ||A p||                   */
#define GSK_BRK_OMEGA 2   /* Bi-CGSTAB: |(t, s)| <= eps_b ||t|| ||s||                         */
#define GSK_BRK_RHO 3     /* Bi-CGSTAB: |(r^, r)| <= eps_b ||r^|| ||r||                       */
#define GSK_BRK_GIVENS 4  /* GMRES: the Hessenberg column to rotate is exactly zero          */

/* Methods for gsk_workspace_bytes */
#define GSK_METHOD_GS 0
#define GSK_METHOD_GMRES 1
#define GSK_METHOD_BICGSTAB 2
#define GSK_METHOD_ARNOLDI 3
#define GSK_METHOD_GMRES_MIXED 4

/* Largest restart length supported by gsk_gmres / gsk_arnoldi. */
#define GSK_MAX_RESTART 64

typedef struct gsk_csr {
    int32_t n;               /* rows = columns, n >= 1                                */
    int64_t nnz;             /* = row_ptr[n] (checked against the device copy)        */
    const int32_t* row_ptr;  /* device [n+1], row_ptr[0] = 0, non-decreasing          */
    const int32_t* col_idx;  /* device [nnz], each in [0, n)                          */
    const double* val;       /* device [nnz]                                          */
} gsk_csr;

/* A matrix as the solvers and gsk_spmv take it. */
#define GSK_MATRIX_CSR 0
#define GSK_MATRIX_STENCIL 1

/* Structured 5-point (nz = 1) or 7-point stencil matrix on an nx x ny x nz grid (x fastest:
 * row i = ix + nx (iy + ny iz), n = nx ny nz; nx, ny >= 2, nz >= 1). coef holds one plane of
 * n FP64 values per stencil position, in the CSR column order -z, -y, -x, centre, +x, +y, +z
 * (7 planes; 5 planes -y, -x, centre, +x, +y when nz = 1): coef[q*n + i] multiplies the q-th
 * neighbour of row i. Neighbours outside the grid are skipped (their plane entries are never
 * read). This is the layout of the paper's 5/7-point central-difference matrices (section
 * 2.1); gsk_stencil_from_csr builds it from a CSR matrix. */
typedef struct gsk_stencil {
    int32_t nx, ny, nz;
    const double* coef;      /* device [7 n] (3D) or [5 n] (2D)                       */
} gsk_stencil;

typedef struct gsk_matrix {
    int32_t kind;            /* GSK_MATRIX_CSR or GSK_MATRIX_STENCIL                  */
    gsk_csr csr;             /* used when kind == GSK_MATRIX_CSR                      */
    gsk_stencil stencil;     /* used when kind == GSK_MATRIX_STENCIL                  */
} gsk_matrix;

typedef struct gsk_options {
    int32_t maxit;              /* iteration cap (GMRES: Arnoldi steps; Bi-CGSTAB:
                                   iterations). Default 10000 (section 2.2).              */
    double breakdown_eps;       /* relative breakdown threshold. Default 1e-16 *
                                   DBL_EPSILON: the paper relaxes AZTEC's brkdown_tol
                                   (= DBL_EPSILON) by about 1e-16 (section 2.2).          */
    const double* stop_weights; /* device [n] or NULL. The stopping test is made on the
                                   GS(2)-scaled system (section 2.2); when the system was
                                   scaled by GS(p) with p != 2, pass the weights
                                   ||a_i||_p/||a_i||_2 written by gsk_gs_scale, and the
                                   test measures ||W (b - A x)|| instead of ||b - A x||.  */
    int32_t check_every;        /* Bi-CGSTAB: iterations enqueued between host status
                                   reads (default 8; 1..256). GMRES reads once per cycle. */
} gsk_options;

typedef struct gsk_info {
    int32_t iters;            /* GMRES: Arnoldi steps; Bi-CGSTAB: iterations (a half-step
                                 exit counts as one)                                       */
    int32_t restarts;         /* GMRES: cycles after the first; Bi-CGSTAB: recurrence
                                 restarts after a failed true-residual check               */
    int32_t status;           /* GSK_CONVERGED / GSK_MAXIT / GSK_BREAKDOWN / GSK_STAGNATED  */
    int32_t half_step;        /* Bi-CGSTAB: 1 if it stopped on ||s|| after half a step      */
    int32_t verify_failures;  /* consecutive failed true-residual checks at the end        */
    int32_t breakdown_test;   /* with GSK_BREAKDOWN: which test fired (GSK_BRK_*), else 0    */
    int32_t fp64_from;        /* mixed-precision Bi-CGSTAB engine: iterations done before the
                                 solve continued in FP64 (0: it never did)                 */
    int32_t reserved;         /* 0                                                         */
    double relres_recursive;  /* last recursive estimate ||W r||/||W r0||                  */
    double relres_true;       /* ||W (b - A x)|| / ||W (b - A x0)|| at return              */
} gsk_info;

/* Fills *opt with the defaults listed above. */
void gsk_default_options(gsk_options* opt);

/* Bytes of device workspace an entry point needs for a system of n rows (m: restart length
 * for GSK_METHOD_GMRES / GSK_METHOD_GMRES_MIXED / GSK_METHOD_ARNOLDI, ignored otherwise).
 * For GSK_METHOD_GMRES_MIXED the figure assumes a 7-point stencil matrix (its FP32 copy
 * lives in the workspace); use gsk_workspace_bytes_for for any other matrix. Returns 0 for
 * invalid arguments. The workspace must be 256-byte aligned; its contents need no
 * initialisation and are garbage afterwards. */
size_t gsk_workspace_bytes(int32_t method, int32_t n, int32_t m);

/* Exact workspace bytes of `method` for matrix *A (host-side checks only; nothing is read
 * from device memory). Returns 0, with the reason in gsk_last_error(), for invalid
 * arguments. */
size_t gsk_workspace_bytes_for(const gsk_matrix* A, int32_t method, int32_t m);

/*
 * GS(p) geometric scaling (section 1; section 2, eq. (2)): for each row i,
 *   nrm_i = ||a_i||_p = (sum_j |a_ij|^p)^(1/p),   a_ij <- a_ij / nrm_i,   b_i <- b_i / nrm_i,
 * so that every row of the scaled matrix has unit Lp-norm. p >= 1 is an integer (p = 2 in
 * the paper's experiments; p = 1 is AZTEC's "row-sum scaling").
 *   A        : input matrix (A->val is read).
 *   b        : device [n] input right-hand side.
 *   val_out  : device [nnz] scaled values (may equal A->val for in-place scaling).
 *   b_out    : device [n] scaled right-hand side (may equal b).
 *   row_norm : device [n] or NULL; receives nrm_i.
 *   stop_weight : device [n] or NULL; receives ||a_i||_p / ||a_i||_2, the stop-test weights
 *              to pass in gsk_options.stop_weights when p != 2 (all ones for p = 2).
 *   ws, ws_bytes : workspace of gsk_workspace_bytes(GSK_METHOD_GS, n, 0) bytes.
 * Errors: GSK_ERR_INVALID_ARG (p < 1, NULL pointers, n < 1), GSK_ERR_ZERO_ROW (some
 * sum_j |a_ij|^p is zero), GSK_ERR_NONFINITE (NaN/Inf in A or b, or a norm that overflows).
 * On GSK_ERR_ZERO_ROW / GSK_ERR_NONFINITE the outputs are unspecified (rows that passed are
 * written, the others are not). Synchronises `stream`.
 */
int gsk_gs_scale(const gsk_csr* A, const double* b, int32_t p, double* val_out, double* b_out,
                 double* row_norm, double* stop_weight, void* ws, size_t ws_bytes,
                 void* stream);

/*
 * y = A x, FP64. Each row is summed in storage order (CSR) or in the CSR column order of the
 * stencil positions (stencil), with every product rounded before it is added, so the result
 * equals a sequential CPU loop without fused multiply-add, and a stencil matrix gives the same
 * bits as the CSR matrix it was packed from. x and y must not overlap. Asynchronous: enqueued
 * on `stream`, no synchronisation. This is the sparse product inside every Krylov step of
 * section 2's solvers.
 */
int gsk_spmv(const gsk_matrix* A, const double* x, double* y, void* stream);

/*
 * Packs a CSR matrix whose pattern is a subset of the 5-point (nz = 1) or 7-point stencil of
 * an nx x ny x nz grid into coefficient planes (gsk_stencil layout). Positions a row does not
 * store get 0. A->n must equal nx ny nz. coef: device [7 n] or [5 n], written.
 * ws, ws_bytes: workspace of gsk_workspace_bytes(GSK_METHOD_GS, n, 0) bytes.
 * Errors: GSK_ERR_INVALID_ARG for bad dimensions, an invalid CSR structure, or an entry that is
 * not a stencil position of its row (or repeats one). Synchronises `stream`.
 */
int gsk_stencil_from_csr(const gsk_csr* A, int32_t nx, int32_t ny, int32_t nz, double* coef,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * m steps of Arnoldi with double classical Gram-Schmidt (section 2: AZTEC's GMRES
 * orthogonalises with a double classical Gram-Schmidt step), started at r0 != 0:
 *   v_1 = r0/||r0||; for j = 1..m: w = A v_j; twice { c = V_j^T w; w -= V_j c; h_{1:j,j} += c };
 *   h_{j+1,j} = ||w||; v_{j+1} = w / h_{j+1,j}.
 * Stops early at a happy breakdown (h_{j+1,j} <= eps_b ||A v_j||, eps_b = 1e-16*DBL_EPSILON).
 *   V : device, column-major n x (m+1) with leading dimension ldv >= n; receives v_1..v_{k+1}
 *       (v_{k+1} only when no breakdown occurred).
 *   H : device, column-major (m+1) x m with leading dimension m+1; receives the Hessenberg
 *       matrix (entries beyond the steps taken are zero).
 *   steps : host int; receives the number of steps k taken (<= m).
 *   ws, ws_bytes : workspace of gsk_workspace_bytes(GSK_METHOD_ARNOLDI, n, m) bytes.
 * 1 <= m <= GSK_MAX_RESTART. Synchronises `stream`.
 */
int gsk_arnoldi(const gsk_matrix* A, const double* r0, int32_t m, double* V, int64_t ldv,
                double* H, int32_t* steps, void* ws, size_t ws_bytes, void* stream);

/*
 * Restarted GMRES(m) (section 2: restarted GMRES with double classical Gram-Schmidt) on
 * A x = b, normally the GS-scaled system.
 *   x   : device [n]; holds x0 on entry (the paper uses x0 = 0, section 2.1) and the
 *         solution on return.
 *   m   : restart length, 1 <= m <= GSK_MAX_RESTART (the paper uses 10).
 *   tol : stop when ||W (b - A x)|| / ||W (b - A x0)|| < tol (section 2.2), verified with the
 *         true residual at the end of a cycle; W from opt->stop_weights (identity if NULL).
 *   opt : NULL for the defaults.
 *   info: host; receives the outcome.
 *   ws, ws_bytes : workspace of gsk_workspace_bytes(GSK_METHOD_GMRES, n, m) bytes.
 * Each Arnoldi step's orthogonalisation coefficients, the Givens rotations and the
 * residual estimate stay on the device; the host reads a small status block once per cycle.
 * Synchronises `stream`.
 */
int gsk_gmres(const gsk_matrix* A, const double* b, double* x, int32_t m, double tol,
              const gsk_options* opt, gsk_info* info, void* ws, size_t ws_bytes, void* stream);

/*
 * GMRES(m) with FP32 Arnoldi cycles and FP64 restarts: iterative refinement in which each
 * correction is one GMRES(m) cycle. The paper's solver is FP64 GMRES (section 2); this form
 * keeps its algorithm and stop test and changes only the storage precision inside a cycle.
 *   - Inside a cycle the matrix values (an FP32 copy the call makes in the workspace), the
 *     basis and w are stored in FP32; products, dot products, the Hessenberg matrix, the
 *     Givens rotations and y are computed in FP64.
 *   - At every restart r = b - A x is computed in FP64 with the caller's matrix and x is
 *     updated in FP64, so the final accuracy is that of FP64 GMRES; `tol` and the stop test
 *     are those of gsk_gmres, verified in FP64.
 *   - A cycle whose FP32 estimate claims convergence that the FP64 residual does not confirm
 *     counts towards STAGNATED only if it did not halve the true residual.
 * Arguments as for gsk_gmres; workspace gsk_workspace_bytes_for(A, GSK_METHOD_GMRES_MIXED, m)
 * bytes (FP32 matrix copy, basis and w: about half the FP64 solver's). info->iters counts
 * Arnoldi steps and info->restarts the FP64 restarts. Synchronises `stream`.
 */
int gsk_gmres_mixed(const gsk_matrix* A, const double* b, double* x, int32_t m, double tol,
                    const gsk_options* opt, gsk_info* info, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * Bi-CGSTAB (section 2: van der Vorst's Bi-CGSTAB) on A x = b, shadow residual r^ = r0.
 * Arguments as for gsk_gmres without m; workspace gsk_workspace_bytes(GSK_METHOD_BICGSTAB,
 * n, 0). All scalars (rho, alpha, omega, beta) stay on the device; the host reads a status
 * block every opt->check_every iterations. Synchronises `stream`.
 */
int gsk_bicgstab(const gsk_matrix* A, const double* b, double* x, double tol,
                 const gsk_options* opt, gsk_info* info, void* ws, size_t ws_bytes,
                 void* stream);

/*
 * Bi-CGSTAB that allocates nothing, for callers that cannot allocate: tight serving loops
 * and harnesses that forbid hipMalloc (it synchronises `stream`, so it is not for use under
 * stream capture). Arguments and results as for gsk_bicgstab, without the workspace: the
 * solver runs in a file-scope device array of gsk_bicgstab_noalloc_max_bytes() bytes
 * (32 MiB), one per GPU the library runs on, held until the process ends. A system whose
 * Bi-CGSTAB workspace (gsk_workspace_bytes(GSK_METHOD_BICGSTAB, n, 0)) exceeds it, about
 * 575,000 rows and more, is rejected with GSK_ERR_WORKSPACE. The call makes no hipMalloc,
 * hipFree, pinned-memory or event allocation: status is read back with a copy into host
 * stack memory and a stream synchronisation per chunk of iterations, and the measurement
 * hook does not time its launches. Results equal gsk_bicgstab's bit for bit.
 * Every call on a GPU uses that GPU's one array: calls that overlap on the same GPU (from
 * several host threads, or on several streams) race and must be serialised by the caller.
 */
int gsk_bicgstab_noalloc(const gsk_matrix* A, const double* b, double* x, double tol,
                         const gsk_options* opt, gsk_info* info, void* stream);
size_t gsk_bicgstab_noalloc_max_bytes(void);

/*
 * Measurement hook (not part of the method). Between gsk_probe_begin(c, k) and gsk_probe_end,
 * every k-th launch of kernel class c made by the solvers is timed: it is launched with a pair
 * of HIP events (hipExtLaunchKernel on the solver's stream, so the events take the dispatch's
 * own start and end times), and it carries
 * a device slot in which it stores its algorithmic HBM bytes if it does work (a launch that
 * returns at once because the solve had already finished leaves it zero and is not counted).
 * Algorithmic bytes per launch, n rows, nnz nonzeros, FP64 values, int32 indices, step j of an
 * Arnoldi cycle (basis columns 0..j):
 *   GMRES_A   12 nnz + 4 (n+1) + 8 n (j+2)   CSR + basis columns 0..j (column j is also the
 *                                            product's source) + write w
 *   GMRES_B   8 n (j+3)                      basis columns 0..j, read and write w
 *   GMRES_C   8 n (j+3)                      basis columns 0..j, read w, write u_{j+1}
 *   BICG_P    12 nnz + 4 (n+1) + 48 n        CSR, r p v r^, write p v (32 n on the first
 *                                            iteration after a start: r r^, write p v)
 *   BICG_S    12 nnz + 4 (n+1) + 24 n        CSR, r v, write t (+8 n with stop weights)
 *   BICG_U    64 n                           r v p x t r^, write x r (+8 n with weights;
 *                                            24 n after a half-step exit)
 *   RESIDUAL  12 nnz + 4 (n+1) + 24..40 n    CSR, x b, write r (and r^ in Bi-CGSTAB), weights
 *   GMRES_X   8 n (k+2)                      k basis columns, read and write x
 * For a stencil matrix the matrix term 12 nnz + 4 (n+1) becomes 8 n per coefficient plane
 * (40 n for 5 points, 56 n for 7). In gsk_gmres_mixed the basis and w terms count 4 bytes per
 * value, the GMRES_A matrix term is that of the FP32 copy (4 n per plane, or 8 nnz + 4 (n+1)),
 * GMRES_X moves 4 n k + 16 n, and RESIDUAL (FP64 matrix, x, b, FP32 u_0) moves the FP64
 * matrix term + 20 n (+ 8 n with weights).
 * Process-wide; not for concurrent use from several host threads. gsk_probe_end
 * synchronises the device.
 */
#define GSK_KCLASS_GMRES_A 1
#define GSK_KCLASS_GMRES_B 2
#define GSK_KCLASS_GMRES_C 3
#define GSK_KCLASS_BICG_P 4
#define GSK_KCLASS_BICG_S 5
#define GSK_KCLASS_BICG_U 6
#define GSK_KCLASS_RESIDUAL 7
#define GSK_KCLASS_GMRES_X 8
/* Batch engine classes (FP64 Bi-CGSTAB engine): the engine samples whole chunks, every k-th
 * chunk is enqueued without its captured graph and each launch of the class in it is timed.
 * Bytes per launch are the BICG_P / BICG_S / BICG_U figures summed over the systems that the
 * launch works on (systems whose solve is at that stage). */
#define GSK_KCLASS_BATCH_P 9
#define GSK_KCLASS_BATCH_S 10
#define GSK_KCLASS_BATCH_U 11

typedef struct gsk_probe_result {
    int64_t launches;       /* launches of the class that were timed                      */
    int64_t busy_launches;  /* of those, launches that did work                           */
    double total_ms;        /* summed event-measured durations of the working timed launches */
    double bytes;           /* summed algorithmic bytes of the working timed launches     */
} gsk_probe_result;

int gsk_probe_begin(int32_t kernel_class, int32_t sample_every);
int gsk_probe_end(gsk_probe_result* out);

/*
 * Measurement hook (not part of the method): the memory ceiling of a streaming kernel's mix of
 * arrays on this device. Times `reps` (1..1000) launches (after one warm-up launch) of a
 * kernel that reads `reads` arrays and writes `writes` arrays of n doubles, one row per thread
 * in 256-row tiles in the solvers' workgroup order, with one tile reduction into a partial and
 * no gathers; *best_ms receives the shortest launch (HIP events). The mixes of the batch engine's
 * passes are supported: (11, 2) P with 7-point planes, (9, 1) S, (6, 2) U, and (1, 0) a plain
 * read, (1, 1) a copy; any other gives GSK_ERR_INVALID_ARG. buf: device memory of at least
 * gsk_stream_mix_bytes(reads, writes, n) bytes (the arrays back to back, then the partials),
 * overwritten. Blocks until the launches have finished.
 */
size_t gsk_stream_mix_bytes(int32_t reads, int32_t writes, int64_t n);
int gsk_stream_mix_ms(int32_t reads, int32_t writes, int64_t n, void* buf, size_t buf_bytes,
                      int32_t reps, float* best_ms, void* stream);

/*
 * Batched Bi-CGSTAB and the solve engine (continuous batching). The paper solves one system
 * at a time (section 2); GS scaling makes every row independent and Bi-CGSTAB needs only
 * products and dot products (section 3 calls it inherently parallel), so many independent
 * systems can share every launch. Each system is solved exactly as gsk_bicgstab solves it
 * (same operations, same per-tile partial sums in the same order), so it returns bit for
 * bit the same x and gsk_info alone, in a batch, or admitted while others run.
 *
 * The engine works in a caller-owned device workspace of gsk_engine_workspace_bytes(max_rows,
 * max_systems) bytes: room for max_rows rows of solver vectors (each system takes its n rows
 * rounded up to a multiple of 256) and max_systems control blocks. A system's matrix (CSR or
 * stencil), b, x and stop weights stay in the caller's device memory, untouched except for
 * x, until the system is reported done. The engine object itself is a host allocation.
 *
 * Time runs in chunks: gsk_engine_run(e, c) enqueues c chunks on the engine's stream, each
 * the residual launch (which starts newly submitted systems and verifies convergence claims)
 * followed by check_every Bi-CGSTAB iterations of every admitted system; systems that are
 * done simply skip. gsk_engine_poll reads every system's status after the last enqueued chunk
 * and retires the finished ones, freeing their rows and slots for new submissions.
 * With flags & GSK_ENGINE_GRAPH the first chunk is captured in a HIP graph and every chunk
 * is a replay of it (needs a non-default stream and an even check_every).
 * An engine is not thread-safe; use one per host thread and stream.
 */
typedef struct gsk_engine gsk_engine;

#define GSK_ENGINE_GRAPH 1
/* gsk_engine_submit: the system did not fit (no free slot or not enough contiguous rows). */
#define GSK_FULL 1

typedef struct gsk_result {
    int64_t tag;        /* the tag given at submission                                    */
    gsk_info info;      /* as gsk_bicgstab would return it; status -1: invalid CSR,
                           -2: zero row, -3: non-finite data (GS stage)                     */
} gsk_result;

typedef struct gsk_engine_usage {
    int32_t active;             /* systems admitted and not yet retired                    */
    int32_t max_systems;
    int64_t max_rows;
    int64_t free_rows;          /* rows not held by any system                             */
    int64_t largest_free_rows;  /* largest system (in rows) that fits now                  */
} gsk_engine_usage;

size_t gsk_engine_workspace_bytes(int64_t max_rows, int32_t max_systems);

/* Errors: GSK_ERR_INVALID_ARG (sizes, check_every out of [1, 256], GRAPH with the default
 * stream or an odd check_every), GSK_ERR_WORKSPACE (NULL, misaligned or too small). */
int gsk_engine_create(void* ws, size_t ws_bytes, int64_t max_rows, int32_t max_systems,
                      int32_t check_every, int32_t flags, void* stream, gsk_engine** out);

/* Admits one system A x = b (normally GS-scaled); x holds x0 and receives the solution.
 * tol and opt as for gsk_bicgstab (opt->check_every is ignored: the engine's applies).
 * Returns GSK_OK, GSK_FULL (nothing changed; retry after a poll has retired systems), or an
 * error for invalid arguments. Enqueues a small initialisation on the engine's stream. */
int gsk_engine_submit(gsk_engine* e, const gsk_matrix* A, const double* b, double* x,
                      double tol, const gsk_options* opt, int64_t tag);

/* Admits one unscaled system with a GS(p) stage (section 2, eq. (2)): the engine's first chunk
 * writes the GS(p)-scaled matrix values to val_out (nnz doubles for CSR, the planes' count
 * for a stencil matrix, same layout as A's values), the scaled right-hand side to b_out [n]
 * and, for p != 2, the stop-test weights ||a_i||_p / ||a_i||_2 to stop_weight_out [n]
 * (required then; ignored for p = 2), all with the arithmetic of gsk_gs_scale. The solve then
 * runs on the scaled system with the GS(2)-metric stop test (section 2.2), exactly as
 * gsk_gs_scale followed by gsk_bicgstab would. opt->stop_weights must be NULL. A zero row or
 * non-finite data ends the system with info.status -2 or -3. Outputs must stay allocated
 * until the system is reported done. */
int gsk_engine_submit_gs(gsk_engine* e, const gsk_matrix* A, const double* b, int32_t p,
                         double* val_out, double* b_out, double* stop_weight_out, double* x,
                         double tol, const gsk_options* opt, int64_t tag);

/*
 * Mixed-precision Bi-CGSTAB engines (GSK_METHOD_BICGSTAB with GSK_PRECISION_MIXED): iterative
 * refinement whose corrections are Bi-CGSTAB runs with FP32 storage of the matrix (a copy the
 * engine writes into the request's mat32) and of r, r^, p, v, t; x, the true residual
 * r = b - A x (with the FP64 matrix) and every sum stay FP64. A run ends at a reduction by
 * inner_reduction of the residual it started from; a refinement step that does not halve the
 * true residual counts towards GSK_STAGNATED. Not in the paper. Rows are handed out in pairs
 * of 256-row tiles.
 *
 * GMRES(m) engines. The same engine runs restarted GMRES(m) with CGS2 Arnoldi (section 2) for
 * many systems at once, in FP64 or with FP32 Arnoldi cycles and FP64 restarts (the iterative
 * refinement of gsk_gmres_mixed). Each system returns bit for bit what gsk_gmres (or
 * gsk_gmres_mixed) returns for it alone. A chunk is one restart cycle: systems start their
 * cycles together at a chunk's start, run up to m Arnoldi steps, and at the chunk's end get
 * x += V y and the true residual (convergence test and the next cycle's start). A system
 * submitted between chunks starts at the next chunk.
 * Rows: a system of n rows takes ceil(n / 256) tiles of 256 rows, rounded up to an even
 * number in a mixed engine (two tiles per workgroup for FP32 data).
 * Workspace: gsk_engine_workspace_bytes_ex; it holds the basis (m+1 columns of max_rows values,
 * 8 or 4 bytes each) and one control block (about 70 KB) per system slot.
 */
#define GSK_PRECISION_FP64 0
#define GSK_PRECISION_MIXED 1

typedef struct gsk_engine_config {
    int64_t max_rows;      /* rows of vectors the engine holds                              */
    int32_t max_systems;   /* system slots                                                  */
    int32_t method;        /* GSK_METHOD_BICGSTAB or GSK_METHOD_GMRES                       */
    int32_t m;             /* GMRES restart length, 1..GSK_MAX_RESTART (ignored otherwise)  */
    int32_t precision;     /* GSK_PRECISION_FP64, or GSK_PRECISION_MIXED: FP32 storage with
                              FP64 iterative refinement (GMRES: FP32 Arnoldi cycles; Bi-CGSTAB:
                              FP32 runs, see inner_reduction)                               */
    int32_t check_every;   /* Bi-CGSTAB: iterations per chunk (1..256, even with
                              GSK_ENGINE_GRAPH); GMRES: ignored (a chunk is one cycle)      */
    int32_t flags;         /* GSK_ENGINE_GRAPH                                              */
    int32_t tile_units;    /* FP64 Bi-CGSTAB: 256-row tiles per workgroup of the streaming
                              launches, 1 or 2 (0 selects 1); a shape choice only, the
                              results are the same bits. Mixed engines use 2, FP64 GMRES 1. */
    double inner_reduction; /* mixed Bi-CGSTAB: a run with FP32 storage ends (and the FP64
                              residual is recomputed) once its estimate has dropped by this
                              factor below the residual it started from, or below tol;
                              0 selects 1e-6; otherwise in (0, 1)                           */
    int32_t run_cap;       /* mixed Bi-CGSTAB: a run with FP32 storage also ends after this
                              many iterations; 0 selects 1000, -1: no cap                   */
    int32_t class_shapes;  /* FP64 Bi-CGSTAB: launch shape per size class, 0 for one shape
                              (tile_units) for every system. Classes: 0 = 2D stencils and
                              CSR matrices, 1 = 3D stencils of fewer than 2^18 rows, 2 = 3D
                              stencils of 2^18 rows or more; bits 4c..4c+3 hold class c's
                              code: 1 = P and S one tile per workgroup, U one tile; 2 = P and
                              S two tiles per workgroup, U one tile; 3 = P and S two tiles,
                              U a unit's two tiles in turn; 0 = the code tile_units selects
                              (2 -> 3, otherwise 1). Each class then has its own launches and
                              rows are handed out in pairs of tiles. A shape choice only:
                              every system returns the same bits under any code.          */
} gsk_engine_config;

/* 0 for an invalid configuration. */
size_t gsk_engine_workspace_bytes_ex(const gsk_engine_config* cfg);

/* As gsk_engine_create, for any configuration. GSK_ENGINE_GRAPH needs a non-default stream;
 * GMRES chunks are captured once per streaming grid size like Bi-CGSTAB chunks. */
int gsk_engine_create_ex(const gsk_engine_config* cfg, void* ws, size_t ws_bytes, void* stream,
                         gsk_engine** out);

/* One system for gsk_engine_submit_ex.
 * gs_p = 0: A and b are already scaled (as for gsk_engine_submit); gs_p >= 1: the GS(p) stage
 * of gsk_engine_submit_gs with its outputs val_out, b_out, stop_weight_out.
 * mat32 (mixed GMRES engines: required; otherwise NULL): device buffer for the FP32 copy of
 * the scaled matrix, which the engine writes in the system's first chunk: for a stencil matrix
 * planes of mat32_ld >= n floats (a multiple of 64 keeps every plane 256-byte aligned), for
 * CSR nnz floats. It must stay allocated until the system is reported done. */
typedef struct gsk_engine_request {
    const gsk_matrix* A;
    const double* b;
    double* x;              /* x0 on entry, the solution when reported done                 */
    double tol;
    const gsk_options* opt; /* nullable; opt->stop_weights must be NULL when gs_p >= 1       */
    int64_t tag;
    int32_t gs_p;
    double* val_out;
    double* b_out;
    double* stop_weight_out;
    float* mat32;
    int64_t mat32_ld;
} gsk_engine_request;

/* Returns GSK_OK, GSK_FULL, or GSK_ERR_INVALID_ARG (also for a mixed engine without mat32). */
int gsk_engine_submit_ex(gsk_engine* e, const gsk_engine_request* r);

/* Enqueues `chunks` chunks (asynchronous). */
int gsk_engine_run(gsk_engine* e, int32_t chunks);

/* Retires the systems finished at the end of the last enqueued chunk. wait != 0 blocks until
 * that chunk has run; wait == 0 returns *n_out = 0 if it has not. At most max_out results are
 * returned per call (the rest stay admitted and are reported by the next poll after another
 * run). */
int gsk_engine_poll(gsk_engine* e, int32_t wait, gsk_result* out, int32_t max_out,
                    int32_t* n_out);

int gsk_engine_get_usage(gsk_engine* e, gsk_engine_usage* u);

/* Synchronises the engine's stream and frees the host object. */
int gsk_engine_destroy(gsk_engine* e);

/* Solves count independent systems in one batch (an engine created in ws, every system
 * submitted, chunks run until all are done). b[i], x[i]: device pointers of system i; info:
 * host array of count. Workspace: gsk_bicgstab_batch_workspace_bytes(count, n) with n the
 * host array of the systems' row counts. */
size_t gsk_bicgstab_batch_workspace_bytes(int32_t count, const int32_t* n);
int gsk_bicgstab_batch(int32_t count, const gsk_matrix* A, const double* const* b,
                       double* const* x, double tol, const gsk_options* opt, gsk_info* info,
                       void* ws, size_t ws_bytes, void* stream);

/* Message for the last error returned on this thread ("" if none). */
const char* gsk_last_error(void);

/* GSK_VERSION of the built library. */
int gsk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSK_H */
