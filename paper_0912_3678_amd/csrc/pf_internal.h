// Internal interface between the host planner (api.cpp) and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "pf.h"
#include <stdint.h>

struct pf_factor_s;

namespace pf {

// Block sizes with kernel instantiations; other m are padded up to the next.
constexpr int kMaxM = 32;

// One level of the recursion: the matrix this level factors and the reduced
// matrix it produces for the next level.
struct LevelArgs {
    int64_t nb;            // block rows of this level's matrix
    int64_t p;             // partitions
    const double *D;       // nb blocks
    const double *Dadd;    // optional second addend of D (reduced levels), or null
    const double *Lo;      // nb-1 blocks
    const double *Up;      // nb-1 blocks (BTRI) or null
    const double *C;       // BABD corner or null
    void *E;               // per block row: inverse of the eliminated pivot block
    void *R;               // per block row: left-separator spike row (BTRI)
    void *Z;               // per block row: left-separator spike column
    void *X;               // per block row: D'^{-1} Up (BTRI)
    double *nD;            // next level: diagonal blocks
    double *nDadd;         // next level: second addend of the diagonal (BTRI)
    double *nLo;           // next level: sub-diagonal blocks
    double *nUp;           // next level: super-diagonal blocks (BTRI)
    double *nC;            // next level: corner (BABD)
    unsigned long long *status;  // packed (level << 40 | block); atomicMin
    void *dump;            // kDumpBytes of scratch that masked stores write into
    const double *zero;    // kZeroBytes of zeros: the target of out-of-range loads
    int level;
    const int64_t *sep;    // explicit partition boundaries (p + 1 entries), or null: balanced
    double tau;            // > 0: a pivot block whose smallest pivot is below tau times its
                           // largest counts as failing (ill-conditioned), besides zero pivots
    unsigned long long *badlist;   // with a list: every failing partition appends its code
    unsigned *badcount;
    int badcap;
};

// Device scratch that receives the stores a lane must not make, and a block
// of zeros that out-of-range loads read instead of real data: the chain
// loops keep every memory operation unconditional and select nothing after a
// load, so their wait counters stay exact.
constexpr size_t kDumpBytes = 64 * 1024;
constexpr size_t kZeroBytes = 16 * 1024;   // >= one 32 x 32 FP64 block

// One level of a solve.
struct SolveArgs {
    int64_t nb, p;
    int32_t nrhs;
    const double *Lo;      // this level's sub-diagonal blocks (forward sweep)
    const void *E, *R, *Z, *X;
    const double *F;       // right-hand sides of this level (ld ldf)
    const double *Fadd;    // optional second addend (reduced levels)
    int64_t ldf;
    double *Y;             // forward: t; backward: x (ld ldy)
    int64_t ldy;
    double *nF;            // next level right-hand side (ld ldn)
    double *nFadd;
    int64_t ldn;
    const double *Xsep;    // backward: next level's solution (ld ldn)
    double *dump;          // kDumpBytes of scratch for masked stores
    const double *zero;    // kZeroBytes of zeros
    const int64_t *sep;    // explicit partition boundaries, or null (as LevelArgs)
};

// Factor launchers, two lane mappings.
// Rows (kernels_rows.hip, M = 1..32): a group of M lanes per partition, lane
// i holding row i of each block.
hipError_t launch_btri_factor(int M, bool f32, const LevelArgs &a, hipStream_t s);
hipError_t launch_babd_factor(int M, bool f32, const LevelArgs &a, hipStream_t s);
// Segments (kernels_seg.hip): M*M/E lanes per partition, E consecutive
// entries of a block row per lane, for the (M, E) pairs seg_ok accepts.
// With sv != NULL (1 <= sv->nrhs <= M) the launch also runs the forward
// sweep of launch_*_fwd for those right-hand sides (factor-and-solve).
bool seg_ok(int M, int E);
// matrix-core factor kernel (finest level, FP64 block tridiagonal, M = 8):
// two partitions per workgroup; the batched form serves work items (table
// entry, partition block) like the other batched factor launches
bool mfma_ok(int kind, int M, bool f32, bool add);
int mfma_partitions_per_wg();
hipError_t launch_mfma_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s);
hipError_t launch_mfma_factor_batch(const LevelArgs *tab, const int4 *work, int nwg, hipStream_t s);
// matrix-core factor kernel for block tridiagonal levels with M = 32 (any
// level; one partition per workgroup; f32: FP32 arithmetic and factors on the
// FP32 matrix-core instruction, else FP64)
hipError_t launch_mfma32_factor(const LevelArgs &a, bool f32, hipStream_t s);
hipError_t launch_mfma32_factor_batch(bool add, bool f32, const LevelArgs *tab, const int4 *work,
                                      int nwg, hipStream_t s);
// the same for M = 16 (sv: also sweep 1..16 right-hand sides forward)
hipError_t launch_mfma16_factor(const LevelArgs &a, const SolveArgs *sv, bool f32, hipStream_t s);
hipError_t launch_mfma16_factor_batch(bool add, bool f32, const LevelArgs *tab, const int4 *work,
                                      int nwg, hipStream_t s);
// matrix-core factor kernel for bidiagonal-plus-corner levels with M = 16
// (any level; one partition per workgroup; sv: also sweep 1..16 right-hand
// sides forward)
hipError_t launch_mfma_babd16_factor(const LevelArgs &a, const SolveArgs *sv, bool f32,
                                     hipStream_t s);
hipError_t launch_mfma_babd16_factor_batch(bool f32, const LevelArgs *tab, const int4 *work,
                                           int nwg, hipStream_t s);
// matrix-core forward sweep / back substitution for M = 16, 32 (FP64 or FP32
// factors): one partition per workgroup, solve32_cols(M, f32, wide64,
// nrhs, parts) right-hand sides each
int solve32_cols(int M, bool f32, bool wide64, int nrhs, int64_t parts);
hipError_t launch_solvet(int M, int kind, bool fwd, bool add, bool f32, const SolveArgs &a,
                         hipStream_t s);
hipError_t launch_solvet_batch(int M, int kind, bool fwd, bool add, bool f32, int cols,
                               const SolveArgs *tab, const int4 *work, int nwg, hipStream_t s);
inline bool solve_tiled(int M, bool) { return M == 16 || M == 32; }
// the FP32 instantiations behind those launchers (kernels_mfma_tiles32.hip)
namespace fp32 {
hipError_t launch_mfma32_factor(const LevelArgs &a, hipStream_t s);
hipError_t launch_mfma32_factor_batch(bool add, const LevelArgs *tab, const int4 *work, int nwg,
                                      hipStream_t s);
hipError_t launch_mfma16_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s);
hipError_t launch_mfma16_factor_batch(bool add, const LevelArgs *tab, const int4 *work, int nwg,
                                      hipStream_t s);
hipError_t launch_mfma_babd16_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s);
hipError_t launch_mfma_babd16_factor_batch(const LevelArgs *tab, const int4 *work, int nwg,
                                           hipStream_t s);
hipError_t launch_solvet(int M, int kind, bool fwd, bool add, const SolveArgs &a, hipStream_t s);
hipError_t launch_solvet_batch(int M, int kind, bool fwd, bool add, int cols, const SolveArgs *tab,
                               const int4 *work, int nwg, hipStream_t s);
}  // namespace fp32
int seg_partitions_per_wg(int M, int E);
hipError_t launch_seg_factor(int kind, int M, int E, bool f32, const LevelArgs &a,
                             const SolveArgs *sv, hipStream_t s);
// Solve launchers (kernels_solve.hip, M = 1..32).
hipError_t launch_btri_fwd(int M, bool f32, const SolveArgs &a, hipStream_t s);
hipError_t launch_btri_bwd(int M, bool f32, const SolveArgs &a, hipStream_t s);
hipError_t launch_babd_fwd(int M, bool f32, const SolveArgs &a, hipStream_t s);
hipError_t launch_babd_bwd(int M, bool f32, const SolveArgs &a, hipStream_t s);

// Batched launches: one launch serves every entry of a device table; work[w]
// = (table entry, partition block, right-hand-side block, unused) for
// workgroup w.  A solve partition block is groups_per_wg(M) partitions, a
// right-hand-side block rhs_chunk(nrhs, parts) columns; a factor work item covers
// groups_per_wg(M) (rows) or seg_partitions_per_wg(M, E) (segments)
// partitions.  Entries of one launch share kind, M, the mapping, precision,
// the ADD variant and (solves) the chunk size.
int groups_per_wg(int M);
// Right-hand-side columns per solve work item (vector-ALU solves): 1, 4, or 8
// for more than four columns when the launch holds at least kWideParts
// partitions (the factor rows are then read half as often; with fewer
// partitions the columns are the launch's parallelism).
constexpr int64_t kWideParts = 8192;
int rhs_chunk(int nrhs, int64_t parts);
hipError_t launch_factor_batch(int kind, int M, bool f32, bool add, const LevelArgs *tab,
                               const int4 *work, int nwg, hipStream_t s);
hipError_t launch_seg_factor_batch(int kind, int M, int E, bool f32, bool add, const LevelArgs *tab,
                                   const int4 *work, int nwg, hipStream_t s);
hipError_t launch_solve_batch(int kind, bool fwd, int M, bool f32, bool add, int KC,
                              const SolveArgs *tab, const int4 *work, int nwg, hipStream_t s);

// Utility kernels (kernels_util.hip).
// Copy m x m blocks into M x M blocks (M >= m); the extra diagonal entries
// are set to `diag` (1 for diagonal blocks, 0 otherwise).
hipError_t launch_pad_blocks(int m, int M, int64_t count, const double *src, double *dst,
                             double diag, hipStream_t s);
// Copy n x nrhs (ld ldsrc) between an m-block and an M-block row layout.
hipError_t launch_pad_rhs(int m, int M, int64_t nb, int32_t nrhs, const double *src,
                          int64_t lds, double *dst, int64_t ldd, bool to_padded,
                          hipStream_t s);
// One system's operands of the residual (see launch_residual).
struct ResidualArgs {
    int kind, m;
    int64_t nb;
    const double *D, *Lo, *Up, *C;
    int nrhs;
    const double *f;
    int64_t ldf;
    const double *x;
    int64_t ldx;
    double *r;
    int64_t ldr;
    unsigned long long *norms, *normA;
};
// block sizes with a grouped (batched) residual launch
bool residual_batched(int m);
// The grouped residual's work units: a system of block size m is cut into
// steps of residual_step_rows(m) rows; workgroup w serves system work[w].x,
// its steps work[w].y .. work[w].z - 1 (at most residual_item_steps()) and
// column chunk work[w].w (64 right-hand sides); systems with live[sys] == 0
// are skipped.  wantA: ||A||_inf of the chunk-0 workgroups into normA;
// write_r: store r (else norms only).
int residual_step_rows(int m);
int residual_item_steps();
hipError_t launch_residual_batch(int m, const ResidualArgs *tab, const int4 *work, int nwg,
                                 const unsigned char *live, bool wantA, bool write_r,
                                 hipStream_t s);
// r = f - A x (FP64; r may be null: norms only) with the max-abs norms of r,
// x, f per right-hand side accumulated into norms[3*c + {0,1,2}], and, when
// normA is not null, ||A||_inf into *normA (ordered uint64 bit patterns of
// non-negative doubles; the caller zeroes them).
hipError_t launch_residual(int kind, int m, int64_t nb, const double *D, const double *Lo,
                           const double *Up, const double *C, int32_t nrhs, const double *f,
                           int64_t ldf, const double *x, int64_t ldx, double *r, int64_t ldr,
                           unsigned long long *norms, unsigned long long *normA, hipStream_t s);
// x += d
// x += d for many systems in one launch (see kb_axpy): per system its
// operands; workgroup w serves system work[w].x, element units work[w].y ..
// work[w].z - 1 of kAxpyUnit elements of its n x nrhs columns
struct AxpyArgs {
    double *x;
    const double *d;
    int64_t n, ldx, ldd;
    int nrhs;
};
constexpr int64_t kAxpyUnit = 65536;
hipError_t launch_axpy_batch(const AxpyArgs *tab, const int4 *work, int nwg,
                             const unsigned char *live, hipStream_t s);
hipError_t launch_axpy(int64_t n, int32_t nrhs, const double *d, int64_t ldd, double *x,
                       int64_t ldx, hipStream_t s);
// Fill count 64-bit words with a value (kernel, capture-safe).
hipError_t launch_ivp_trapezoid(int m, int64_t steps, const double *L, double h, const double *g,
                                const double *y0, double *D, double *Lo, double *C, double *f,
                                hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long v,
                           hipStream_t s);
hipError_t launch_band_to_btri(int64_t n, int kl, int ku, const double *ab, int64_t ldab,
                               int m, double *D, double *Lo, double *Up, hipStream_t s);
hipError_t launch_abd_to_btri(int m, int64_t N, int qa, const double *Ba, const double *S,
                              const double *R, const double *Bb, double *D, double *Lo,
                              double *Up, hipStream_t s);

// Timing of one launch from inside its dispatch packet: a launcher whose
// next kernel launch finds these events set launches it with
// hipExtLaunchKernel, which stamps the kernel's own start and end into them,
// and clears them (kernels_util.hip holds the thread-local instance).
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchTiming &launch_timing();

// Handle helpers for the request scheduler (api.cpp): factor a new handle
// and solve in one go on a stream, release without a host wait, and read the
// status word of a handle whose work is complete.
// Device memory of a handle: alloc / free callbacks (null: stream-ordered
// hipMallocAsync / hipFreeAsync).
struct Allocator {
    pf_alloc_fn alloc = nullptr;
    pf_free_fn free = nullptr;
    void *ctx = nullptr;
};
// al: the allocator of the new handle (null: the one pf_set_allocator set);
// setup_ms (may be null): host time of the handle's set-up and allocation
int factor_new_solve(const pf_matrix *A, const pf_opts *opts, hipStream_t s, int nrhs,
                     const double *f, int64_t ldf, double *x, int64_t ldx, pf_factor_s **out,
                     const Allocator *al = nullptr, double *setup_ms = nullptr);
void destroy_async(pf_factor_s *F);
// Factor-and-solve with all device memory carved from [base, base + cap)
// (pf_factor_solve_static); and the HIP error kept for pf_last_hip_error.
int factor_solve_in(const pf_matrix *A, const pf_opts *opts, char *base, size_t cap, int nrhs,
                    const double *f, int64_t ldf, double *x, int64_t ldx, hipStream_t s,
                    pf_info *info);
void note_hip_error(hipError_t e);
// Refinement (PF_FP32_IR) as separate queued steps for the request
// scheduler, in the order of pf_solve's loop: the residual and its norms into
// host words (3 nrhs + 1, pinned), eta from them, a correction solve with
// x += d; and a solve with stored factors without refinement.
int ir_queue_residual(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, const double *x,
                      int64_t ldx, hipStream_t s, unsigned long long *host);
int ir_queue_correction(pf_factor_s *F, int nrhs, double *x, int64_t ldx, hipStream_t s);
double ir_eta(const unsigned long long *host, int nrhs);
const pf_opts &handle_opts(const pf_factor_s *F);
int solve_queued(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, double *x, int64_t ldx,
                 hipStream_t s);
int status_nosync(pf_factor_s *F, pf_info *info);

// Options of a PF_FLAG_AUTOTUNE factorization (tune.cpp): the cached choice
// for A's shape class, tuning on A first when there is none.
int tuned_opts(const pf_matrix *A, const pf_opts &o, int nrhs, hipStream_t s, pf_opts *out);

// work decomposition of a solve launch (batched solves): partitions per
// workgroup and right-hand-side columns per workgroup (M = 16 and 32 with
// FP64 factors: the matrix-core kernels)
inline int solve_groups_per_wg(int M, bool f32) { return solve_tiled(M, f32) ? 1 : groups_per_wg(M); }
inline int solve_cols(int M, bool f32, bool wide64, int nrhs, int64_t parts)
{
    return solve_tiled(M, f32) ? solve32_cols(M, f32, wide64, nrhs, parts)
                               : rhs_chunk(nrhs, parts);
}

}  // namespace pf
