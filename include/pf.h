/*
 * pf.h -- partition-method factor-and-solve for structured linear systems on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: the "parallel factorization" A = F T G of Amodio & Brugnano,
 * "Parallel factorizations in numerical analysis", Sec. 2, eqs. (parpart),
 * (parfact)-(parG), (parblock) with the LU local factorization, the reduced
 * matrices of eqs. (redmatr) and (redmatr1), and the ODE-IVP reading of
 * Sec. 3 (eqs. (D), (recur), (pups)).  The unknowns are split into
 * partitions separated by single separator blocks; every partition is
 * eliminated independently (one group of lanes per partition), the small
 * reduced system on the separators is assembled from the partitions'
 * contributions and solved by applying the same method to it recursively,
 * and the partitions are then back-substituted independently.
 *
 * All functions are plain C.  Pointers named "device" must be HIP device
 * memory; everything else is host memory.  Streams are hipStream_t passed as
 * void* (NULL = the default stream).
 *
 * Matrix storage (caller-owned DEVICE memory, FP64, never modified):
 *   an m x m block is column-major: entry (i,j) at blk[i + j*m]; a block
 *   array is a contiguous sequence of blocks (block k at offset k*m*m).
 *   PF_BTRI (block tridiagonal; m == 1 is scalar tridiagonal):
 *       D[k]  = A(k,k)    for k = 0..nb-1
 *       Lo[k] = A(k+1,k)  for k = 0..nb-2
 *       Up[k] = A(k,k+1)  for k = 0..nb-2          (C must be NULL)
 *   PF_BABD (lower block bidiagonal plus a top-right corner block: BABD
 *       matrices from one-step ODE-BVP methods with non-separated boundary
 *       conditions, circulant-like matrices after a row permutation, and the
 *       discrete IVP of Sec. 3 with C = 0; the form after eq. (redmatr1)):
 *       D[k]  = A(k,k)    for k = 0..nb-1  (D[0] = B0, D[k+1] = R_k)
 *       Lo[k] = A(k+1,k)  for k = 0..nb-2  (S_k)
 *       C     = A(0,nb-1)                  (B1; Up must be NULL)
 * Right-hand sides and solutions are n x nrhs column-major (n = m*nb) with
 * a leading dimension >= n, in DEVICE memory.
 *
 * Errors: 0 = success; negative = invalid argument number -k (checked on
 * the host before any work is queued); positive = a PF_E* code below.
 * Numeric problems found on the device (an exactly zero pivot) are reported
 * by pf_sync_status / pf_solve with info != NULL.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { PF_BTRI = 0, PF_BABD = 1 } pf_kind;

/* PF_FP64: every elimination in FP64.
 * PF_FP32_IR: the finest-level eliminations in FP32 (factors stored in
 * FP32), the reduced separator systems in FP64, and FP64 iterative
 * refinement on the FP64 residual r = f - A x until the normwise backward
 * error eta <= tol. */
typedef enum { PF_FP64 = 0, PF_FP32_IR = 1 } pf_prec;

enum {
    PF_OK = 0,
    PF_ESINGULAR = 1,   /* exactly zero pivot inside a pivot block            */
    PF_ENOCONV = 2,     /* refinement stagnated, hit max_refine, or met a
                           non-finite residual                              */
    PF_ENOMEM = 3,      /* a device allocation ran out of memory             */
    PF_EHIP = 4,        /* a HIP runtime call failed (any other error of an
                           allocation included): pf_last_hip_error        */
    PF_EUNSUPPORTED = 5,/* block size beyond what the library instantiates   */
    PF_ETOOBIG = 6      /* pf_factor_solve_static: the system's factor memory
                           exceeds the static workspace (256 MiB)           */
};

enum {
    PF_FLAG_ETA = 1,       /* pf_solve in FP64 also computes eta (one residual pass)  */
    PF_FLAG_MAP_ROWS = 2,  /* factor every level with the row lane mapping (M lanes per
                              partition, lane i holds row i of each block) instead of
                              the defaults: the segment mapping (M*M/E lanes per
                              partition, E block entries per lane: E = 1 for m <= 8,
                              4 for m = 16) with matrix-core products at the finest
                              level of FP64 PF_BTRI matrices with m = 8, and for FP64
                              PF_BTRI matrices with m = 32 matrix-core products on
                              every level (other m = 32 levels use rows).  The
                              mappings differ only in rounding.                      */
    PF_FLAG_MAP_TILES = 4, /* reserved (the segment mapping is the default)         */
    PF_FLAG_AUTOTUNE = 8,  /* pf_factor / pf_batch_create take block_rows,
                              coarse_rows, lane_entries and the mapping from the
                              autotuner's cache for the system's shape class,
                              tuning on this matrix first when the class is new
                              (see pf_autotune)                                      */
    PF_FLAG_MAP_SEGMENTS = 16, /* the finest level of an FP64 PF_BTRI matrix with
                              m = 8 (after padding) runs its block products on the
                              matrix cores by default (v_mfma_f64_16x16x4f64,
                              two partitions per wave); this flag, or lane_entries
                              > 0, keeps it on the segment mapping.  The mappings
                              differ only in rounding.                               */
    PF_FLAG_ENLARGE = 32   /* pf_factor, PF_BTRI: the enlarged reduced system of Sec. 2
                              (the modified factorization after eq. (redmatr)).  Where a
                              partition's elimination meets a pivot block that is
                              singular (a zero pivot) or ill-conditioned (its
                              smallest pivot below 2^-40 of its largest, 2^-20 for
                              FP32 factors), the elimination stops before it and
                              that block row joins the separators, so it enters the
                              reduced system, where the neighbours' contributions
                              are added to it; the level is planned again with the
                              enlarged separator list (partitions may be empty) and
                              factored again, up to 32 passes.  pf_factor then
                              synchronizes `stream`; the handle keeps the separator
                              lists (pf_factor_level reports the enlarged p), and
                              pf_refactor / pf_factor_solve reuse them (a pivot block
                              that fails there is reported as PF_ESINGULAR).
                              pf_factor_bytes does not include the enlargement.
                              The finest level of m = 8 then runs on the segment
                              mapping.  PF_BABD: the reduced matrix of eq. (redmatr1)
                              keeps each separator's own diagonal block, so moving a
                              failing block there cannot cure it; pf_factor makes one
                              pass, which also flags ill-conditioned pivot blocks
                              (PF_ESINGULAR with the first one).                    */
};

typedef struct {
    int32_t kind;       /* pf_kind                                            */
    int32_t m;          /* block size, 1 <= m <= 32                           */
    int64_t nb;         /* number of block rows (= unknown blocks), >= 2      */
    const double *D;    /* device, nb blocks                                  */
    const double *Lo;   /* device, nb-1 blocks                                */
    const double *Up;   /* device, nb-1 blocks (PF_BTRI) or NULL (PF_BABD)    */
    const double *C;    /* device, 1 block (PF_BABD) or NULL (PF_BTRI)        */
} pf_matrix;

typedef struct {
    int32_t partitions; /* partitions p of the finest level; 0 = planner.
                           PF_BTRI: 1 <= p <= (nb+1)/2;
                           PF_BABD: 1 <= p <= (nb-1)/2                        */
    int32_t prec;       /* pf_prec                                            */
    int32_t max_refine; /* PF_FP32_IR iteration cap; <= 0 means 10           */
    int32_t block_rows; /* blocks per partition at the finest level when
                           partitions == 0; 0 = the planner's table (Sec. 2
                           leaves p free), doubled up to 64 while the level
                           keeps at least 16384 partitions (m > 1)            */
    int32_t flags;      /* PF_FLAG_*                                          */
    int32_t coarse_rows;/* blocks per partition on the reduced levels; 0 = table */
    int32_t lane_entries;/* finest level, segment lane mapping: block entries per
                           lane (1: one entry; 2: m = 8; 4: m = 16); 0 = planner */
    double tol;         /* PF_FP32_IR target eta; <= 0 means 1e-12            */
} pf_opts;

typedef struct {
    int32_t status;       /* PF_OK or a PF_E* code                           */
    int32_t refine_iters; /* refinement corrections applied (PF_FP32_IR)     */
    int32_t bad_level;    /* level of the first zero pivot (0 = input)        */
    int32_t reserved;
    int64_t bad_block;    /* block row of that pivot at that level, else -1  */
    double eta;           /* normwise backward error
                             ||f-Ax||/(||A|| ||x|| + ||f||) (inf-norms, max
                             over right-hand sides); -1 when not computed    */
} pf_info;

typedef struct pf_factor_s *pf_factor_t;

/* ---- device memory and HIP errors ----------------------------------------
 * Ownership of factor memory (the factors, the reduced systems, the status
 * words and the solve workspace of a handle; the one allocation of a batch):
 * it is allocated through the allocator set here, and the handle or batch
 * gives it back through the matching free when it is destroyed.  Default
 * (and after pf_set_allocator(NULL, NULL, NULL)): stream-ordered
 * hipMallocAsync / hipFreeAsync on the stream the handle was created on.
 *   alloc(bytes, stream, ctx) returns device memory of at least `bytes`
 *     bytes, 256-byte aligned, usable by work queued on `stream` (a
 *     hipStream_t), or NULL when it has none (the call then fails with
 *     PF_ENOMEM);
 *   free(ptr, bytes, stream, ctx) takes back a block alloc returned; work
 *     on `stream` that uses the block may still be queued, so the allocator
 *     must order its reuse after that work (hipFreeAsync and PyTorch's
 *     caching allocator both do).
 * Each handle and batch keeps the allocator that was current when it was
 * created (its blocks go back to that one).  Setting the allocator is not
 * synchronized with other host threads creating handles.  Small argument
 * tables of batches (a few bytes per partition block) and the plan of the IVP
 * driver stay on hipMalloc / hipMallocAsync.  Returns 0, or -1 / -2 when only
 * one of the two functions is given. */
typedef void *(*pf_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*pf_free_fn)(void *ptr, size_t bytes, void *stream, void *ctx);
int pf_set_allocator(pf_alloc_fn alloc, pf_free_fn free, void *ctx);

/* The hipError_t of the most recent HIP call of the calling thread that made
 * a library call fail with PF_EHIP (or PF_ENOMEM: hipErrorOutOfMemory);
 * 0 if none has failed. */
int pf_last_hip_error(void);

/* Factor A (eqs. (parfact), (parblock) with the LU variant, applied
 * recursively to the reduced matrix (redmatr)/(redmatr1)).
 * The handle keeps pointers to A's arrays (PF_FP32_IR refinement and the
 * forward solve read them): A must stay valid and unmodified until
 * pf_destroy.  Work is queued on `stream`; numeric status is read by
 * pf_sync_status.  Returns 0, -k for invalid argument k, PF_ENOMEM, PF_EHIP
 * or PF_EUNSUPPORTED. */
int pf_factor(const pf_matrix *A, const pf_opts *opts, void *stream, pf_factor_t *out);

/* Factor again, in the handle's memory, after the values of A's arrays
 * changed (same pointers, same structure): the numeric refactorization of
 * repeated solves (Newton steps, time stepping).  Allocates nothing.
 * Returns 0 or PF_EHIP; numeric status as for pf_factor. */
int pf_refactor(pf_factor_t F, void *stream);

/* Per-kernel timing with HIP events recorded around every launch of the
 * handle's factor and solve calls (on the stream they run on).  Off by
 * default.  pf_profile_read synchronizes and returns the number of entries
 * of the most recent factor/refactor and solve calls (up to max are copied):
 * phase 0 = factor, 1 = forward sweep, 2 = back substitution, 3 = factor
 * with the forward sweep fused (pf_factor_solve); level = the recursion
 * level; ms = the launch's duration. */
int pf_profile_enable(pf_factor_t F, int enable);
int pf_profile_read(pf_factor_t F, int32_t max, int32_t *phase, int32_t *level, float *ms);

/* Solve A x = f with the factors (the F, T and G solves of Sec. 2: parallel
 * forward sweeps, the recursive reduced solve, parallel back substitution;
 * for PF_FP32_IR also the FP64 refinement loop).  f and x may be the same
 * buffer.  If info != NULL the call synchronizes `stream` and fills it;
 * otherwise it is fully asynchronous (PF_FP64) -- PF_FP32_IR always
 * synchronizes once per refinement step to test eta. */
int pf_solve(pf_factor_t F, int32_t nrhs, const double *f, int64_t ldf, double *x,
             int64_t ldx, void *stream, pf_info *info);

/* Factor-and-solve: factor A again in the handle's memory (as pf_refactor:
 * same pointers, new values) and solve A x = f, as pf_refactor followed by
 * pf_solve.  Where every level runs on the tile mapping and 1 <= nrhs <= m
 * (padded block size), each level is factored and its right-hand sides are
 * swept forward in one pass (the F solve of Sec. 2 alongside the
 * factorization), which saves one pass over the factors per level.  The
 * factors stay in the handle for later pf_solve calls.  nrhs = 0 only
 * refactors.  Arguments, errors and synchronization as for pf_solve. */
int pf_factor_solve(pf_factor_t F, int32_t nrhs, const double *f, int64_t ldf, double *x,
                    int64_t ldx, void *stream, pf_info *info);

/* Factor-and-solve that allocates no device memory, for callers that cannot
 * call hipMalloc (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same plan and kernels as pf_factor
 * followed by pf_factor_solve (results equal bit for bit), with every device
 * byte of the factorization -- factors, reduced systems, status words and
 * solve workspace -- carved from one static device array of 256 MiB that
 * each GPU the library runs on holds until the process ends.  No handle is
 * returned: the factors live in that array until the next call on the same
 * GPU overwrites them.  Calls that overlap on one GPU (other streams, other
 * host threads, before an earlier call's work has finished) share the array
 * and race: order them on one stream or synchronize between them.  The
 * stream must belong to the current device.  A, opts, f, ldf, x, ldx and
 * info as for pf_factor and pf_factor_solve (nrhs = 0 only factors);
 * PF_FLAG_AUTOTUNE is refused (argument 2: tuning allocates).  With info ==
 * NULL and PF_FP64 the call is asynchronous and issues kernels only (it can
 * be captured into a graph); otherwise it synchronizes `stream`.  Returns 0,
 * -k for invalid argument k, PF_ETOOBIG when the system needs more than the
 * array holds, PF_EHIP, or the numeric status. */
int pf_factor_solve_static(const pf_matrix *A, const pf_opts *opts, int32_t nrhs, const double *f,
                           int64_t ldf, double *x, int64_t ldx, void *stream, pf_info *info);

/* Autotuner: time pf_factor_solve of A (nrhs right-hand sides, f = 1) on
 * `stream` for candidate launch shapes -- finest-level chain length
 * (block_rows 4..32), its lane mapping (every segment width with a kernel
 * for the block size, and rows) and the reduced levels' chain length
 * (coarse_rows 2..6) -- and return the fastest as *best (with its median
 * time in *best_ms, may be NULL).  Precision, tolerance and the other
 * fields come from *base (may be NULL).  The choice is also cached for the
 * system's shape class (kind, block size, precision, nb to half an octave,
 * right-hand-side bucket), where PF_FLAG_AUTOTUNE finds it.  Allocates and
 * frees its own scratch; synchronizes `stream`.  Returns 0, -k for invalid
 * argument k, PF_ENOMEM or PF_EHIP. */
int pf_autotune(const pf_matrix *A, const pf_opts *base, int32_t nrhs, void *stream,
                pf_opts *best, float *best_ms);
/* Forget every cached autotuner choice. */
void pf_autotune_clear(void);

/* ---- batches of independent systems ---------------------------------------
 * The partitions of many systems run side by side: every system's
 * per-partition work of one level and phase goes into one kernel launch per
 * launch variant (kind, block size, precision), the partitions of all
 * systems spread over the workgroups of that launch.  The factor and solve
 * sequence of the whole batch is recorded once into a HIP graph and replayed;
 * the launches of each block size form a branch of their own, so different
 * block sizes run side by side.
 *
 * Partitions (Sec. 2): with opts->block_rows and opts->partitions 0, the
 * systems of one kind and block size m > 1 whose chain length the autotuner
 * leaves open share a finest-level chain length: the longest, from the
 * one-system default up to 64 blocks, that leaves at least 16384 partitions
 * in their grouped launch (a batch has parallelism to spare where one system
 * does not, and longer chains shrink the reduced levels).  A small batch keeps
 * the one-system plan, and pf_batch_factor's handles report the plan used
 * (pf_factor_level).
 *
 * pf_batch_create: A, nrhs, f, ldf, x, ldx are HOST arrays of nsys entries
 * describing DEVICE buffers (layouts as for pf_factor / pf_solve; nrhs[i] may
 * be 0).  The batch keeps these pointers: pf_batch_run factors every A[i] as
 * it is at that moment and solves into x[i] from f[i], so the caller may
 * change the values (not the pointers) between runs.  One device allocation
 * holds all factors and workspaces.  Synchronizes `stream` once.  Returns 0,
 * -k for invalid argument k, PF_ENOMEM, PF_EHIP or PF_EUNSUPPORTED. */
typedef struct pf_batch_s *pf_batch_t;
int pf_batch_create(int32_t nsys, const pf_matrix *A, const pf_opts *opts,
                    const int32_t *nrhs, const double *const *f, const int64_t *ldf,
                    double *const *x, const int64_t *ldx, void *stream, pf_batch_t *out);

/* Replay the batch after the work queued so far on `stream`; later work on
 * `stream` sees the solutions.  With info == NULL and PF_FP64 the call is
 * asynchronous; otherwise it synchronizes and fills info[0..nsys) per system
 * (PF_FP32_IR refines every system of the batch together until each meets
 * tol or stops converging).  Returns 0 or the first nonzero per-system
 * status.  Runs of one batch must not overlap. */
int pf_batch_run(pf_batch_t B, void *stream, pf_info *info);

/* Per-launch timing of a batch: the batch's factor and solve launches are
 * issued once more without the graph (the same work: the solutions are
 * written as by pf_batch_run; PF_FP32_IR runs no refinement here), each
 * grouped launch timed by HIP events that its dispatch stamps on the stream
 * it runs on.  Fills up to max entries of out, sets *count to the number of
 * grouped launches and returns 0 (or -k for invalid argument k, PF_EHIP);
 * synchronizes.
 * phase: 0 factor, 1 forward sweep, 2 back substitution; level: recursion
 * level; m: the block size the kernel runs at (padded); mapping (factor
 * launches): > 0 segment width, 0 rows, < 0 a matrix-core kernel; rows:
 * block rows of all its systems; rhs_rows: block rows x right-hand sides
 * (solve launches); ms: the launch's duration. */
typedef struct {
    int32_t phase, level, kind, m, f32, mapping;
    int64_t rows, rhs_rows;
    int32_t workgroups;
    float ms;
} pf_launch_info;
int pf_batch_profile(pf_batch_t B, void *stream, int32_t max, pf_launch_info *out,
                     int32_t *count);

/* Hand out the factor of system i as a handle (pf_solve, pf_refactor,
 * pf_destroy work on it); each system can be handed out once.  The handle
 * shares the batch's allocation, which lives until the batch and every
 * handed-out handle are destroyed. */
int pf_batch_factor(pf_batch_t B, int32_t i, pf_factor_t *out);

/* Release the batch (synchronizes its internal stream). */
void pf_batch_destroy(pf_batch_t B);

/* One-shot batch: create, run, destroy.  factors (may be NULL) is in/out,
 * one entry per system: an entry that is non-NULL on entry is the caller's
 * existing factor of A[i] (same kind, m, nb and precision; from pf_factor, a
 * batch or this call) and system i is solved with it, in the batch's grouped
 * solve launches, without being factored again (the handle's solve
 * workspace grows on its own stream if nrhs[i] needs it); an entry that is
 * NULL on entry is factored by the batch and its new factor is handed out
 * in it, for the caller to destroy.  An existing factor must not be used by
 * other work while the call runs.  Argument errors as for pf_batch_create,
 * and -10 for an existing factor that does not match A[i] or opts->prec.
 * Synchronizes `stream`. */
int pf_solve_batch(int32_t nsys, const pf_matrix *A, const pf_opts *opts,
                   const int32_t *nrhs, const double *const *f, const int64_t *ldf,
                   double *const *x, const int64_t *ldx, void *stream,
                   pf_factor_t *factors, pf_info *info);

/* Device bytes pf_factor allocates for A with these options (admission
 * control), and that pf_solve adds per right-hand side. */
size_t pf_factor_bytes(const pf_matrix *A, const pf_opts *opts);
size_t pf_solve_bytes_per_rhs(const pf_matrix *A, const pf_opts *opts);

/* Synchronize the factor's stream and report the device-side status of the
 * factorization (zero pivots). */
int pf_sync_status(pf_factor_t F, pf_info *info);

/* The FP64 residual of the refinement (PF_FP32_IR) and of PF_FLAG_ETA, and
 * the norms of the normwise backward error eta = ||r|| / (||A|| ||x|| + ||f||)
 * (infinity norms) those tests take: r = f - A x for nrhs columns, with A of
 * eq. (syst)'s block forms as in pf_matrix (device arrays).  f, x: device,
 * n x nrhs, ld ldf / ldx >= n = m nb; r: device, n x nrhs, ld ldr >= n, or
 * NULL for the norms only.  norms: host, 3 nrhs + 1 doubles, filled on
 * return: ||r_c||, ||x_c||, ||f_c|| for column c at 3c .. 3c+2, then ||A||.
 * Queued on `stream` (NULL = the default stream) behind its work, with a
 * small stream-ordered scratch of 3 nrhs + 1 words from the allocator;
 * synchronizes `stream`.  Returns 0, -k for invalid argument k, PF_ENOMEM or
 * PF_EHIP. */
int pf_residual(const pf_matrix *A, int32_t nrhs, const double *f, int64_t ldf, const double *x,
                int64_t ldx, double *r, int64_t ldr, void *stream, double *norms);

/* Release the factor's device memory (synchronizes its stream first). */
void pf_destroy(pf_factor_t F);

const char *pf_strerror(int code);

/* ---- plan inspection (host) ------------------------------------------- */
/* Number of levels of the recursion, and for level l its kind, block count
 * and partition count. */
int pf_factor_levels(pf_factor_t F);
int pf_factor_level(pf_factor_t F, int level, int32_t *kind, int64_t *nb, int64_t *p);

/* The level plan pf_factor would use, computed on the host without any
 * device work: returns the number of levels L (or a negative argument
 * error) and fills up to max_levels entries of kinds/nbs/ps (any may be
 * NULL).  Level 0 is A itself; level l+1 is the reduced matrix of level l
 * (p-1 blocks for PF_BTRI, p+1 for PF_BABD); the last level has p = 1. */
int pf_plan(const pf_matrix *A, const pf_opts *opts, int32_t max_levels, int32_t *kinds,
            int64_t *nbs, int64_t *ps);

/* Block size the kernels run at: m rounded up to a power of two (the matrix
 * is padded with identity diagonal entries when it differs from m). */
int pf_factor_block_size(pf_factor_t F);

/* Copy the reduced system that level `level` produced for level+1 into host
 * buffers (FP64, blocks column-major, of the pf_factor_block_size): PF_BTRI gives the (p-1)-block block
 * tridiagonal matrix of eq. (redmatr) (D with the two neighbours'
 * contributions summed, Lo, Up); PF_BABD gives the (p+1)-block BABD of
 * eq. (redmatr1) (D, Lo, C in Up's place).  Synchronizes. */
int pf_factor_export_reduced(pf_factor_t F, int level, double *D, double *Lo, double *Up);

/* ---- structure mapping (device kernels, stream-ordered) ----------------- */
/* Banded matrix (kl sub-, ku super-diagonals; LAPACK band storage: A(i,j) at
 * ab[ku + i - j + j*ldab], ldab >= kl+ku+1) -> PF_BTRI blocks with block size
 * m = max(kl,ku), the block form of a banded matrix in Sec. 2.  n must be a
 * multiple of m.  D, Lo, Up are device outputs of n/m, n/m-1, n/m-1 blocks. */
int pf_band_to_btri(int64_t n, int32_t kl, int32_t ku, const double *ab, int64_t ldab,
                    double *D, double *Lo, double *Up, void *stream);

/* ABD matrix from a one-step method with separated boundary conditions
 * (Sec. 3): qa rows Ba (qa x m) at t0, N step rows [S_k R_k] (m x 2m,
 * S and R as block arrays), qb = m - qa rows Bb (qb x m) at t_N.  Rows are
 * regrouped into N+1 block rows of m rows (row 0 = [Ba; last qb rows of
 * step 0]; row k = [first qa rows of step k-1; last qb rows of step k];
 * row N = [first qa rows of step N-1; Bb]), which is block tridiagonal.
 * Ba, Bb are column-major with leading dimensions qa, qb.  Outputs: N+1, N,
 * N blocks. */
int pf_abd_to_btri(int32_t m, int64_t N, int32_t qa, const double *Ba, const double *S,
                   const double *R, const double *Bb, double *D, double *Lo, double *Up,
                   void *stream);

/* ---- linear initial value problems (Sec. 3) -----------------------------
 * y' = L y + g(t), y(t0) = y0 (L constant, m x m), discretized by the
 * trapezoid rule with `steps` steps of size h: the lower block bidiagonal
 * system of eq. (My) in the bidiagonal-plus-corner form with a zero corner:
 * D[0] = I, D[n] = I - h/2 L (n >= 1), Lo[n-1] = -(I + h/2 L), C = 0,
 * f[0] = y0, f[n] = h/2 (g_{n-1} + g_n).  L: device, column-major; g:
 * device, steps+1 samples g(t0 + n h) of m entries each (sample n at
 * g + n*m); y0: device, m entries.  Outputs (device, caller-allocated): D
 * steps+1 blocks, Lo steps blocks, C one block, f (steps+1)*m entries.
 * Returns 0, -k for invalid argument k, or PF_EHIP. */
int pf_ivp_trapezoid_system(int32_t m, int64_t steps, const double *L, double h, const double *g,
                            const double *y0, double *D, double *Lo, double *C, double *f,
                            void *stream);

/* A plan for time-parallel solutions of such IVPs with a fixed shape: m,
 * a coarse mesh of p sub-intervals of N steps each (N >= 2), options (may be
 * NULL; partitions is replaced by p).  Holds the eq. (My) system arrays and
 * the factor handle, allocated here on `stream` (stream-ordered; the plan
 * keeps using that stream by default).  Returns 0, -k for invalid argument
 * k, PF_ENOMEM or PF_EHIP. */
typedef struct pf_ivp_s *pf_ivp_t;
int pf_ivp_create(int32_t m, int64_t p, int64_t N, const pf_opts *opts, void *stream,
                  pf_ivp_t *out);
/* Solve one IVP with a plan, as pf_ivp_solve describes: builds the system
 * for L, [t0, T], g, y0 into the plan's arrays, then factors and solves it
 * (pf_factor_solve on the plan's handle).  Allocates nothing.  stream NULL =
 * the plan's stream.  Synchronization and errors as for pf_factor_solve. */
int pf_ivp_run(pf_ivp_t I, const double *L, double t0, double T, const double *g,
               const double *y0, double *y, void *stream, pf_info *info);
void pf_ivp_destroy(pf_ivp_t I);

/* Time-parallel solution of that IVP on [t0, T] over a coarse mesh of p
 * sub-intervals of N steps each (Sec. 3): h = (T - t0) / (p N), and the p
 * partitions of the factorization are the sub-intervals.  The finest level
 * then solves the p local problems with zero initial values (eq. (D)) and
 * their fundamental blocks w_i, the reduced system gives the initial values
 * y_{0i} (eqs. (redsys), (recur); solved by the same method, recursively,
 * rather than by the sequential recursion), and the back substitution is the
 * parallel update (eq. (pups)).  g, y0 as for pf_ivp_trapezoid_system (p*N+1
 * samples); y: device output of p*N+1 vectors (y_n at y + n*m).  N >= 2.
 * opts may be NULL (its partitions field is replaced by p; PF_FP64 or
 * PF_FP32_IR).  A one-shot pf_ivp_create + pf_ivp_run + pf_ivp_destroy:
 * allocates the system arrays on `stream` (stream-ordered) and frees them
 * before returning; synchronizes `stream`.  info may be NULL.
 * Returns 0, -k for invalid argument k, PF_ENOMEM, PF_EHIP or the numeric
 * status (PF_ESINGULAR). */
int pf_ivp_solve(int32_t m, const double *L, double t0, double T, int64_t p, int64_t N,
                 const double *g, const double *y0, double *y, const pf_opts *opts, void *stream,
                 pf_info *info);

/* ---- serving: continuous batching under a device-memory budget ----------
 * A request factors A and solves for f (or solves with a factor kept from an
 * earlier request) into x.  Requests are admitted in arrival order as memory
 * (the budget, counted with pf_factor_bytes / pf_solve_bytes_per_rhs) and
 * in-flight slots free up -- a request that does not fit waits while later
 * ones that fit go ahead -- and run concurrently on the server's streams;
 * least recently used kept factors that no pending request needs are
 * evicted to make room.  Scheduling happens inside submit / poll / wait /
 * stats; only pf_server_wait blocks.  PF_FP64 or PF_FP32_IR: a refined
 * request queues its FP32 solve and first residual at admission, and each
 * poll whose residual norms have arrived (pinned host words behind an event)
 * queues the next correction or ends the request -- the same steps, tests
 * and kernels as pf_solve's refinement, without a host wait.  Requests on
 * one kept factor share its residual workspace, so a refined request on it
 * runs only after the one before has finished refining.  Not thread-safe:
 * one host thread drives a server. */
typedef struct pf_server_s *pf_server_t;

typedef struct {
    pf_matrix A;        /* device arrays, valid until the request completes, and while
                           a factor kept with keep = 1 may be used (it points to
                           them; PF_FP32_IR repeats read them for the residual) */
    int32_t nrhs;       /* >= 1                                                */
    int32_t keep;       /* 1: keep the factor resident for later requests     */
    const double *f;    /* device, n x nrhs, ld ldf                            */
    int64_t ldf;
    double *x;          /* device, n x nrhs, ld ldx                            */
    int64_t ldx;
    int64_t factor;     /* -1: factor A; else the ticket of a request with keep = 1
                           whose factor solves this one (same A)               */
    void *after;        /* stream whose work queued so far produces A and f: an event
                           recorded on it at submission orders the request after
                           that work (NULL = the default stream)               */
} pf_request;

typedef struct {
    size_t budget, used;          /* bytes                                     */
    int64_t queued, inflight, resident, completed, evictions;
    double setup_ms_max, setup_ms_total;    /* host time of new requests' handle
                                               set-up and allocation           */
    double launch_ms_max, launch_ms_total;  /* host time of requests' launches
                                               (set-up included)              */
} pf_server_info;

/* budget_bytes: device memory the server may hold; max_inflight: running
 * requests at once (0 = 8); nstreams: concurrent streams (0 = 4, default
 * priority).  opts: as for pf_factor (prec PF_FP64 or PF_FP32_IR; -2 for
 * another). */
int pf_server_create(size_t budget_bytes, const pf_opts *opts, int32_t max_inflight,
                     int32_t nstreams, pf_server_t *out);
/* Queue a request; returns its ticket.  PF_ENOMEM if it can never fit. */
int pf_server_submit(pf_server_t S, const pf_request *req, int64_t *ticket);
/* 1 and the request's status in *info when it is done, else 0. */
int pf_server_poll(pf_server_t S, int64_t ticket, pf_info *info);
/* Block until the request is done; returns its status. */
int pf_server_wait(pf_server_t S, int64_t ticket, pf_info *info);
/* Submission (host clock), start and completion (device events) times of a
 * request in ms since the server's creation; -1 while unknown.  Returns 1
 * when the request is done. */
int pf_server_times(pf_server_t S, int64_t ticket, double *submit_ms, double *start_ms,
                    double *done_ms);
/* Allocate `bytes` (<= budget) of device memory once, ahead of the
 * requests (a server's start-up): the server carves request memory from it
 * with a sub-allocator of its own (best fit, coalescing; a range freed on one
 * stream goes to another only behind an event wait), so no request's
 * allocation reaches the driver, whose mappings of fresh device memory have
 * cost hundreds of milliseconds of host time inside single requests.  What
 * does not fit falls back to the server's memory pool (release threshold =
 * the budget).  Once per server (-3 after that); blocks the host for the
 * allocation.  Returns 0, -k, PF_ENOMEM or PF_EHIP. */
int pf_server_reserve(pf_server_t S, size_t bytes);
/* Drop a kept factor (after the requests queued on it). */
int pf_server_release(pf_server_t S, int64_t factor);
int pf_server_stats(pf_server_t S, pf_server_info *st);
/* Wait for all work and free everything. */
void pf_server_destroy(pf_server_t S);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
