// Bandwidth-bound helper kernels: FP64 residual and norms (refinement and
// the backward-error gate), padding of block sizes without an instantiation,
// the structure mappings of Sec. 2 (banded and ABD -> block tridiagonal) and
// the trapezoid discretization of a linear IVP (Sec. 3).
#include "pf_internal.h"

#include <type_traits>

namespace pf {
namespace {

__device__ __forceinline__ unsigned long long dbits(double v)
{
    return (unsigned long long)__double_as_longlong(v);
}

// *p = max(*p, v) for ordered bit patterns of non-negative doubles, skipping
// the atomic when the value already there is at least v: maxima only grow,
// so a stale read can cost an atomic but never lose one, and the many
// workgroups of a reduction that finish together mostly read instead of
// contending for the same few words
__device__ __forceinline__ void max_bits(unsigned long long *p, double v)
{
    const unsigned long long b = dbits(v);
    if (b > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, b);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// max over the 256 threads of a workgroup (waves reduce with shuffles, then
// one LDS exchange); the result is valid in thread 0
__device__ __forceinline__ double block_max(double v, double *sh)
{
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) v = sh[k] > v ? sh[k] : v;
    return v;
}

// Grid-stride loops over rows with a bounded grid, and one atomic per
// workgroup and norm: the atomics to the few norm words stay few.  A thread
// owns one row and CH right-hand sides (blockIdx.y = the chunk of columns):
// each entry of A is read once per CH columns, so many right-hand sides do
// not multiply the reads of A.  Per column the sum runs in the same order
// for every CH (f, then D, Lo, Up / C by column).
template <int CH, int MT>
__global__ __launch_bounds__(256) void k_residual(int kind, int m_rt, int64_t nb,
                                                  const double *__restrict__ D,
                                                  const double *__restrict__ Lo,
                                                  const double *__restrict__ Up,
                                                  const double *__restrict__ C, int nrhs,
                                                  const double *__restrict__ f, int64_t ldf,
                                                  const double *__restrict__ x, int64_t ldx,
                                                  double *__restrict__ r, int64_t ldr,
                                                  unsigned long long *norms,
                                                  unsigned long long *normA)
{
    const int m = MT ? MT : m_rt;   // block size: compile-time where instantiated
    const bool wantA = normA != nullptr && blockIdx.y == 0;   // ||A||_inf in the first chunk
    const int64_t n = (int64_t)m * nb;
    const int64_t mm = (int64_t)m * m;
    const int c0 = blockIdx.y * CH;
    const int nc = nrhs - c0 < CH ? nrhs - c0 : CH;
    // columns of the chunk, clamped to existing ones (loads stay in bounds
    // and branch-free; only the first nc are stored and reduced)
    int64_t cx[CH], cf[CH], cr[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int64_t cc = c0 + (c < nc ? c : nc - 1);
        cx[c] = cc * ldx;
        cf[c] = cc * ldf;
        cr[c] = cc * ldr;
    }
    double mr[CH], mx[CH], mf[CH], ma = 0.0;
#pragma unroll
    for (int c = 0; c < CH; ++c) mr[c] = mx[c] = mf[c] = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
         row += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = row / m;
        const int i = (int)(row - k * m);
        double s[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            s[c] = f[row + cf[c]];
            mf[c] = fmax(mf[c], fabs(s[c]));
        }
        // s -= blk(i, :) xb(:, c) for every column of the chunk
        // (a partial unroll: loads of several columns in flight without
        // spilling the CH accumulators)
        constexpr int UF = CH >= 16 ? 4 : 8;
        double sa = 0.0;   // sum of |A(row, :)|
        auto apply = [&](const double *blk, const double *xb) {
#pragma unroll UF
            for (int j = 0; j < (MT ? MT : m); ++j) {
                const double a = blk[(int64_t)j * m];
                sa += fabs(a);
#pragma unroll
                for (int c = 0; c < CH; ++c) s[c] = fma(-a, xb[j + cx[c]], s[c]);
            }
        };
        apply(D + k * mm + i, x + k * m);
        if (k > 0) apply(Lo + (k - 1) * mm + i, x + (k - 1) * m);
        if (kind == 0 && k + 1 < nb) apply(Up + k * mm + i, x + (k + 1) * m);
        if (kind == 1 && k == 0) apply(C + i, x + (nb - 1) * m);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (r && c < nc) r[row + cr[c]] = s[c];
            mr[c] = fmax(mr[c], fabs(s[c]));
            mx[c] = fmax(mx[c], fabs(x[row + cx[c]]));
        }
        ma = fmax(ma, sa);
    }
    __shared__ double sh[4];
    if (wantA) {   // uniform per workgroup
        const double a = block_max(ma, sh);
        if (threadIdx.x == 0) max_bits(normA, a);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const double a = block_max(mr[c], sh);
        const double b = block_max(mx[c], sh);
        const double d = block_max(mf[c], sh);
        if (threadIdx.x == 0 && c < nc) {
            max_bits(norms + 3 * (c0 + c) + 0, a);
            max_bits(norms + 3 * (c0 + c) + 1, b);
            max_bits(norms + 3 * (c0 + c) + 2, d);
        }
    }
}

// The residual r = f - A x and the norms of eta on the matrix cores (FP64
// v_mfma_f64_16x16x4f64), for block sizes MB = 4, 8, 16, 32.
//
// A step is S = max(16, MB) consecutive rows (one block row for MB = 32);
// its rows of A touch the window of S + 2 MB columns from the block column
// before its first block row to the one after its last.  Per row tile of 16
// rows the window's A entries are the A operands of KS = (S + 2 MB) / 4
// steps (K index of step p and lane group g: window column 4p + g; entries
// outside the block diagonals zero), the x rows of the window for one tile
// of 16 right-hand sides the B operands, and r = f - acc comes out in the
// result layout (lane (n, g): rows 4q + g of the tile, column n); the steps
// run as two accumulator chains (even and odd) added at the end.
//
// A wave walks a run of consecutive steps for one column tile and keeps the
// x window in registers: the next step's window is this one shifted by S
// rows, so per step only S new rows of x are loaded and x comes from memory
// once per run (plus a window's halo at the run's start), A and f once, r
// is written once.  The loads of a step (A, the new x rows, f) are
// independent and issued together.  The BABD corner C (block row 0 against
// x[nb-1]) is a further chain in the step holding row 0.  ||A||_inf
// (wantA): per row of the tile-0 runs, the sum of |A| over its window entries
// and the corner, summed across the four lane groups.
//
// Per column of the chunk the wave keeps its running maxima of |r|, |x|,
// |f| in its own LDS row (entry (3J + t) 16 + n); the workgroup combines its
// waves' rows and posts one maximum per column and norm.
constexpr int kResCT = 4;     // column tiles per chunk (64 right-hand sides)
constexpr int kResRun = 8;    // steps per run

struct ResShared {
    double col[4][3 * kResCT * 16];
    double a[4];
};

__device__ __forceinline__ void res_begin(ResShared &sh, double &ma)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int e = lane; e < 3 * kResCT * 16; e += 64) sh.col[wv][e] = 0.0;
    ma = 0.0;
}

// the workgroup's waves, then one maximum per column and norm
__device__ __forceinline__ void res_end(const ResidualArgs &a, int chunk, bool wantA,
                                        ResShared &sh, double ma)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (wantA) {
        ma = wave_max(ma);
        if (lane == 0) sh.a[wv] = ma;
    }
    __syncthreads();
    const int cb = chunk * 16 * kResCT;
    for (int e = threadIdx.x; e < 3 * kResCT * 16; e += blockDim.x) {
        const int J = e / 48, t = (e / 16) % 3, col = cb + 16 * J + (e & 15);
        if (col < a.nrhs) {
            const double v =
                fmax(fmax(sh.col[0][e], sh.col[1][e]), fmax(sh.col[2][e], sh.col[3][e]));
            max_bits(a.norms + 3 * col + t, v);
        }
    }
    if (wantA && threadIdx.x == 0)
        max_bits(a.normA, fmax(fmax(sh.a[0], sh.a[1]), fmax(sh.a[2], sh.a[3])));
}

// The runs of steps s0 .. s1 - 1 x the column tiles of the chunk: unit u
// (run u / nt, tile u % nt), the workgroup's waves taking every fourth unit
// (the waves on one run take its tiles together, sharing A in the cache).
template <int MB>
__device__ __forceinline__ void res_item(const ResidualArgs &a, int64_t s0, int64_t s1, int chunk,
                                         bool wantA, bool write_r, ResShared &sh, double &ma)
{
    typedef double v4 __attribute__((ext_vector_type(4)));
    constexpr int S = MB > 16 ? MB : 16;          // rows per step
    constexpr int TI = S / 16;                     // row tiles per step
    constexpr int KS = (S + 2 * MB) / 4;           // window steps
    constexpr int KN = S / 4;                      // new window steps per step
    constexpr int OWN = MB / 4;                    // first window step of the step's own rows
    constexpr int KC = MB / 4;                     // steps of the corner chain
    constexpr int SH = MB == 4 ? 2 : MB == 8 ? 3 : MB == 16 ? 4 : 5;
    constexpr int64_t MM = (int64_t)MB * MB;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int kind = a.kind, nrhs = a.nrhs;
    const int64_t nb = a.nb, N = (int64_t)MB * nb;
    const double *__restrict__ D = a.D;
    const double *__restrict__ Lo = a.Lo;
    const double *__restrict__ Up = a.Up;
    const double *__restrict__ C = a.C;
    const int64_t ldf = a.ldf, ldx = a.ldx, ldr = a.ldr;
    const int cb = chunk * (16 * kResCT);
    const int nt = min(kResCT, (nrhs - cb + 15) / 16);   // column tiles of this chunk
    const int64_t runs = (s1 - s0 + kResRun - 1) / kResRun;
    for (int64_t u = wv; u < runs * nt; u += 4) {
        const int64_t sa = s0 + (u / nt) * kResRun, se = min(sa + kResRun, s1);
        const int J = (int)(u % nt);
        const int c0 = cb + 16 * J;
        const bool act = c0 + n < nrhs;
        const int64_t cc = act ? c0 + n : c0;    // an existing column (loads in bounds)
        const double *__restrict__ xc = a.x + cc * ldx;
        const double *__restrict__ fc = a.f + cc * ldf;
        // window row p of the step at row0: x rows row0 - MB + 4p + g
        auto xload = [&](int64_t row0, int p) -> double {
            const int64_t j0 = row0 - MB + 4 * p;   // uniform; a multiple of 4
            return (act && j0 >= 0 && j0 < N) ? xc[j0 + g] : 0.0;
        };
        double b[KS];
#pragma unroll
        for (int p = 0; p < KS; ++p) b[p] = xload(sa * S, p);
        for (int64_t st = sa; st < se; ++st) {
            const int64_t row0 = st * S;
            if (st > sa) {
#pragma unroll
                for (int p = 0; p < KS - KN; ++p) b[p] = b[p + KN];
#pragma unroll
                for (int p = KS - KN; p < KS; ++p) b[p] = xload(row0, p);
            }
            const int64_t kw = (row0 >> SH) - 1;   // block column of the window's start
            const bool corner = kind == 1 && row0 == 0;
            double mr = 0.0, mx = 0.0, mf = 0.0;
#pragma unroll
            for (int I = 0; I < TI; ++I) {
                // this lane's row i = row0 + 16I + n in block row ki: step p
                // reads D, Lo or Up of block row ki by kc - ki, column
                // (4p & (MB - 1)) + g of the block
                const int64_t i = row0 + 16 * I + n, ki = i >> SH;
                const bool rowok = i < N;
                const int64_t lane_off = (i & (MB - 1)) + (int64_t)g * MB;
                const double *pD = D + ki * MM + lane_off;
                const double *pL = Lo + (ki > 0 ? ki - 1 : 0) * MM + lane_off;
                const double *pU = kind == 0 ? Up + ki * MM + lane_off : nullptr;
                double av[KS], fv[4];
#pragma unroll
                for (int p = 0; p < KS; ++p) {
                    const int64_t kc = kw + ((4 * p) >> SH);
                    const int64_t co = (int64_t)((4 * p) & (MB - 1)) * MB;
                    const int64_t d = kc - ki;
                    double v = 0.0;
                    if (rowok && kc >= 0 && kc < nb) {
                        if (d == 0) v = pD[co];
                        else if (d == -1) v = pL[co];
                        else if (d == 1 && kind == 0) v = pU[co];
                    }
                    av[p] = v;
                }
                const int64_t rt = row0 + 16 * I + g;   // rows rt + 4q of the result
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    fv[q] = (act && rt + 4 * q < N) ? fc[rt + 4 * q] : 0.0;
                // the corner's A operand: C(i, 4p + g) for rows of block row 0
                auto c_at = [&](int p) -> double {
                    return i < MB ? C[i + (int64_t)(4 * p + g) * MB] : 0.0;
                };
                if (wantA && J == 0) {
                    double sa_ = 0.0;
#pragma unroll
                    for (int p = 0; p < KS; ++p) sa_ += fabs(av[p]);
                    if (corner)
#pragma unroll
                        for (int p = 0; p < KC; ++p) sa_ += fabs(c_at(p));
                    sa_ += __shfl_xor(sa_, 16, 64);
                    sa_ += __shfl_xor(sa_, 32, 64);
                    ma = fmax(ma, sa_);
                }
                v4 acc0 = v4{0.0, 0.0, 0.0, 0.0}, acc1 = v4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int p = 0; p + 1 < KS; p += 2) {
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], b[p], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p + 1], b[p + 1], acc1, 0, 0, 0);
                }
                if constexpr (KS % 2)
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[KS - 1], b[KS - 1], acc0, 0, 0, 0);
                if (corner) {
#pragma unroll
                    for (int p = 0; p < KC; ++p) {
                        const double bc = act ? xc[(nb - 1) * MB + 4 * p + g] : 0.0;
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(c_at(p), bc, acc0, 0, 0, 0);
                    }
                }
                const v4 acc = acc0 + acc1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t row = rt + 4 * q;
                    if (act && row < N) {
                        const double rv = fv[q] - acc[q];
                        if (write_r) a.r[row + cc * ldr] = rv;
                        mr = fmax(mr, fabs(rv));
                        mf = fmax(mf, fabs(fv[q]));
                    }
                }
            }
            // the step's own rows of x: window steps OWN .. OWN + KN - 1
#pragma unroll
            for (int p = OWN; p < OWN + KN; ++p) mx = fmax(mx, fabs(b[p]));
            // column n's maxima over the four lane groups, into the wave's row
            double v[3] = {mr, mx, mf};
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                v[t] = fmax(v[t], __shfl_xor(v[t], 16, 64));
                v[t] = fmax(v[t], __shfl_xor(v[t], 32, 64));
                double &cell = sh.col[wv][(3 * J + t) * 16 + n];
                if (g == 0) cell = fmax(cell, v[t]);
            }
        }
    }
}

// steps of S rows in a system (see res_item)
__host__ __device__ constexpr int res_step_rows(int m) { return m > 16 ? m : 16; }
constexpr int kResItemSteps = 4 * kResRun;   // steps per workgroup item

// one system: workgroup b takes items b, b + gridDim.x, ... of kResItemSteps
// steps; blockIdx.y = the chunk of 64 right-hand sides
template <int MB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MB > 16 ? 2 : MB > 8 ? 3 : 4)))
void k_residual_mma(ResidualArgs a)
{
    __shared__ ResShared sh;
    double ma;
    res_begin(sh, ma);
    const bool wantA = a.normA != nullptr && blockIdx.y == 0;
    const int64_t steps = ((int64_t)MB * a.nb + res_step_rows(MB) - 1) / res_step_rows(MB);
    for (int64_t s0 = (int64_t)blockIdx.x * kResItemSteps; s0 < steps;
         s0 += (int64_t)gridDim.x * kResItemSteps)
        res_item<MB>(a, s0, min(s0 + kResItemSteps, steps), blockIdx.y, wantA, a.r != nullptr,
                     sh, ma);
    res_end(a, blockIdx.y, wantA, sh, ma);
}

// a batch: workgroup w serves system work[w].x, steps work[w].y .. work[w].z
// - 1 in chunk work[w].w; systems whose live flag is 0 are skipped; wantA
// and write_r as flags (bit 0, bit 1)
template <int MB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MB > 16 ? 2 : MB > 8 ? 3 : 4)))
void kb_residual_mma(const ResidualArgs *tab, const int4 *work, const unsigned char *live,
                     int flags)
{
    __shared__ ResShared sh;
    const int4 w = work[blockIdx.x];
    if (!live[w.x]) return;   // uniform per workgroup
    const ResidualArgs a = tab[w.x];
    const bool wantA = (flags & 1) && a.normA != nullptr && w.w == 0;
    double ma;
    res_begin(sh, ma);
    res_item<MB>(a, w.y, w.z, w.w, wantA, (flags & 2) != 0, sh, ma);
    res_end(a, w.w, wantA, sh, ma);
}

// x += d for the systems of a batch in one launch: workgroup w serves
// system work[w].x, the elements work[w].y .. work[w].z - 1 of its n x nrhs
// columns taken as one range (element e: row e mod n, column e / n), in
// units of kAxpyUnit elements (work[w].y, .z are unit indices); systems whose
// live flag is 0 are skipped
__global__ __launch_bounds__(256) void kb_axpy(const AxpyArgs *tab, const int4 *work,
                                               const unsigned char *live)
{
    const int4 w = work[blockIdx.x];
    if (!live[w.x]) return;
    const AxpyArgs a = tab[w.x];
    const int64_t total = a.n * a.nrhs;
    const int64_t e0 = (int64_t)w.y * kAxpyUnit, e1 = min((int64_t)w.z * kAxpyUnit, total);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int64_t c = e / a.n, i = e - c * a.n;
        a.x[i + c * a.ldx] += a.d[i + c * a.ldd];
    }
}

__global__ void k_axpy(int64_t n, const double *__restrict__ d, int64_t ldd,
                       double *__restrict__ x, int64_t ldx)
{
    const int c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i + c * ldx] += d[i + c * ldd];
}

__global__ void k_fill_u64(unsigned long long *p, int64_t count, unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_pad_blocks(int m, int M, int64_t count, const double *__restrict__ src,
                             double *__restrict__ dst, double diag)
{
    const int64_t MM = (int64_t)M * M, mm = (int64_t)m * m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count * MM;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / MM;
        const int rem = (int)(e - k * MM);
        const int j = rem / M, i = rem - j * M;
        double v;
        if (i < m && j < m) v = src[k * mm + i + (int64_t)j * m];
        else v = (i == j) ? diag : 0.0;
        dst[e] = v;
    }
}

__global__ void k_pad_rhs(int m, int M, int64_t nb, const double *__restrict__ src, int64_t lds,
                          double *__restrict__ dst, int64_t ldd, int to_padded)
{
    const int c = blockIdx.y;
    const int64_t nP = (int64_t)M * nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nP;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / M;
        const int i = (int)(e - k * M);
        if (to_padded) {
            dst[e + c * ldd] = (i < m) ? src[k * m + i + c * lds] : 0.0;
        } else if (i < m) {
            dst[k * m + i + c * ldd] = src[e + c * lds];
        }
    }
}

// A(r, c) from LAPACK band storage, zero outside the band.
__device__ __forceinline__ double band_at(int64_t n, int kl, int ku, const double *ab,
                                          int64_t ldab, int64_t r, int64_t c)
{
    if (r < 0 || c < 0 || r >= n || c >= n) return 0.0;
    if (r - c > kl || c - r > ku) return 0.0;
    return ab[(ku + r - c) + c * ldab];
}

__global__ void k_band_to_btri(int64_t n, int kl, int ku, const double *__restrict__ ab,
                               int64_t ldab, int m, double *D, double *Lo, double *Up)
{
    const int64_t nb = n / m, mm = (int64_t)m * m;
    const int64_t total = nb * mm;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / mm;
        const int rem = (int)(e - k * mm);
        const int j = rem / m, i = rem - j * m;
        D[e] = band_at(n, kl, ku, ab, ldab, k * m + i, k * m + j);
        if (k + 1 < nb) {
            Lo[e] = band_at(n, kl, ku, ab, ldab, (k + 1) * m + i, k * m + j);
            Up[e] = band_at(n, kl, ku, ab, ldab, k * m + i, (k + 1) * m + j);
        }
    }
}

// Row regrouping of an ABD matrix (separated boundary conditions) into a
// block tridiagonal one; see pf_abd_to_btri.
__global__ void k_abd_to_btri(int m, int64_t N, int qa, const double *__restrict__ Ba,
                              const double *__restrict__ S, const double *__restrict__ R,
                              const double *__restrict__ Bb, double *D, double *Lo, double *Up)
{
    const int qb = m - qa;
    const int64_t mm = (int64_t)m * m;
    const int64_t total = (N + 1) * mm;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / mm;
        const int rem = (int)(e - k * mm);
        const int j = rem / m, i = rem - j * m;
        double dv;
        if (i < qa) dv = (k == 0) ? Ba[i + (int64_t)j * qa] : R[(k - 1) * mm + i + (int64_t)j * m];
        else dv = (k == N) ? Bb[(i - qa) + (int64_t)j * qb] : S[k * mm + i + (int64_t)j * m];
        D[e] = dv;
        if (k < N) {
            Lo[e] = (i < qa) ? S[k * mm + i + (int64_t)j * m] : 0.0;   // A(k+1, k)
            Up[e] = (i < qa) ? 0.0 : R[k * mm + i + (int64_t)j * m];  // A(k, k+1)
        }
    }
}

// The linear IVP y' = L y + g(t), y(t0) = y0, discretized by the trapezoid
// rule with stepsize h over `steps` steps, as the lower block bidiagonal
// system of Sec. 3, eq. (My): y_0 = y0, then for n >= 1
//   (I - h/2 L) y_n - (I + h/2 L) y_{n-1} = h/2 (g_{n-1} + g_n),
// stored as the bidiagonal-plus-corner form with a zero corner.
__global__ void k_ivp_trapezoid(int m, int64_t steps, const double *__restrict__ L, double h,
                                const double *__restrict__ g, const double *__restrict__ y0,
                                double *D, double *Lo, double *C, double *f)
{
    const int64_t mm = (int64_t)m * m;
    const int64_t total = (steps + 1) * mm;
    const double hh = 0.5 * h;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / mm;
        const int rem = (int)(e - k * mm);
        const int j = rem / m, i = rem - j * m;
        const double id = (i == j) ? 1.0 : 0.0, l = L[rem];
        D[e] = (k == 0) ? id : id - hh * l;
        if (k < steps) Lo[e] = -(id + hh * l);   // A(k+1, k)
        if (k == 0) C[rem] = 0.0;
        if (j == 0) f[k * m + i] = (k == 0) ? y0[i] : hh * (g[(k - 1) * m + i] + g[k * m + i]);
    }
}

// workgroups for the reductions: enough to stream HBM, few atomics
inline unsigned grid_reduce(int64_t work, int block)
{
    int64_t g = (work + block - 1) / block;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (unsigned)g;
}

inline unsigned grid1(int64_t work, int block)
{
    int64_t g = (work + block - 1) / block;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

LaunchTiming &launch_timing()
{
    static thread_local LaunchTiming t;
    return t;
}

hipError_t launch_residual(int kind, int m, int64_t nb, const double *D, const double *Lo,
                           const double *Up, const double *C, int32_t nrhs, const double *f,
                           int64_t ldf, const double *x, int64_t ldx, double *r, int64_t ldr,
                           unsigned long long *norms, unsigned long long *normA, hipStream_t s)
{
    const int64_t n = (int64_t)m * nb;
    if (nrhs < 1) return hipSuccess;
    if (m == 4 || m == 8 || m == 16 || m == 32) {
        const ResidualArgs a{kind, m, nb, D, Lo, Up, C, nrhs, f, ldf, x, ldx, r, ldr, norms, normA};
        // one workgroup per item (as the batched launch): the grid's waves
        // all have their loads in flight at once
        const int64_t steps = (n + res_step_rows(m) - 1) / res_step_rows(m);
        int64_t wg = (steps + kResItemSteps - 1) / kResItemSteps;
        if (wg > (1 << 30)) wg = 1 << 30;
        const dim3 grid((unsigned)wg, (nrhs + 16 * kResCT - 1) / (16 * kResCT));
        switch (m) {
        case 4: hipLaunchKernelGGL((k_residual_mma<4>), grid, dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_residual_mma<8>), grid, dim3(256), 0, s, a); break;
        case 16: hipLaunchKernelGGL((k_residual_mma<16>), grid, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((k_residual_mma<32>), grid, dim3(256), 0, s, a); break;
        }
        return hipGetLastError();
    }
    // columns per thread: one, four, or eight (A read once per chunk); the
    // block sizes of the workloads get a fully unrolled row loop
    auto go = [&](auto ch, auto mt) {
        constexpr int CH = decltype(ch)::value, MT = decltype(mt)::value;
        hipLaunchKernelGGL((k_residual<CH, MT>), dim3(grid_reduce(n, 256), (nrhs + CH - 1) / CH),
                           dim3(256), 0, s, kind, m, nb, D, Lo, Up, C, nrhs, f, ldf, x, ldx, r,
                           ldr, norms, normA);
        return hipGetLastError();
    };
    auto by_m = [&](auto ch) {
        switch (m) {
        case 4: return go(ch, std::integral_constant<int, 4>{});
        case 8: return go(ch, std::integral_constant<int, 8>{});
        case 16: return go(ch, std::integral_constant<int, 16>{});
        case 32: return go(ch, std::integral_constant<int, 32>{});
        default: return go(ch, std::integral_constant<int, 0>{});
        }
    };
    if (nrhs == 1) return by_m(std::integral_constant<int, 1>{});
    if (nrhs <= 4) return by_m(std::integral_constant<int, 4>{});
    return by_m(std::integral_constant<int, 8>{});
}

bool residual_batched(int m) { return m == 4 || m == 8 || m == 16 || m == 32; }
int residual_step_rows(int m) { return res_step_rows(m); }
int residual_item_steps() { return kResItemSteps; }

hipError_t launch_residual_batch(int m, const ResidualArgs *tab, const int4 *work, int nwg,
                                 const unsigned char *live, bool wantA, bool write_r,
                                 hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    const int flags = (wantA ? 1 : 0) | (write_r ? 2 : 0);
    switch (m) {
    case 4: hipLaunchKernelGGL((kb_residual_mma<4>), dim3(nwg), dim3(256), 0, s, tab, work, live, flags); break;
    case 8: hipLaunchKernelGGL((kb_residual_mma<8>), dim3(nwg), dim3(256), 0, s, tab, work, live, flags); break;
    case 16: hipLaunchKernelGGL((kb_residual_mma<16>), dim3(nwg), dim3(256), 0, s, tab, work, live, flags); break;
    case 32: hipLaunchKernelGGL((kb_residual_mma<32>), dim3(nwg), dim3(256), 0, s, tab, work, live, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, int32_t nrhs, const double *d, int64_t ldd, double *x,
                       int64_t ldx, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy, dim3(grid1(n, 256), nrhs), dim3(256), 0, s, n, d, ldd, x, ldx);
    return hipGetLastError();
}

hipError_t launch_axpy_batch(const AxpyArgs *tab, const int4 *work, int nwg,
                             const unsigned char *live, hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_axpy, dim3(nwg), dim3(256), 0, s, tab, work, live);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long v,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(grid1(count, 256)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_pad_blocks(int m, int M, int64_t count, const double *src, double *dst,
                             double diag, hipStream_t s)
{
    hipLaunchKernelGGL(k_pad_blocks, dim3(grid1(count * M * M, 256)), dim3(256), 0, s, m, M,
                       count, src, dst, diag);
    return hipGetLastError();
}

hipError_t launch_pad_rhs(int m, int M, int64_t nb, int32_t nrhs, const double *src,
                          int64_t lds, double *dst, int64_t ldd, bool to_padded,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_pad_rhs, dim3(grid1((int64_t)M * nb, 256), nrhs), dim3(256), 0, s, m,
                       M, nb, src, lds, dst, ldd, to_padded ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_band_to_btri(int64_t n, int kl, int ku, const double *ab, int64_t ldab,
                               int m, double *D, double *Lo, double *Up, hipStream_t s)
{
    hipLaunchKernelGGL(k_band_to_btri, dim3(grid1(n * m, 256)), dim3(256), 0, s, n, kl, ku, ab,
                       ldab, m, D, Lo, Up);
    return hipGetLastError();
}

hipError_t launch_ivp_trapezoid(int m, int64_t steps, const double *L, double h, const double *g,
                                const double *y0, double *D, double *Lo, double *C, double *f,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_ivp_trapezoid, dim3(grid1((steps + 1) * m * m, 256)), dim3(256), 0, s, m,
                       steps, L, h, g, y0, D, Lo, C, f);
    return hipGetLastError();
}

hipError_t launch_abd_to_btri(int m, int64_t N, int qa, const double *Ba, const double *S,
                              const double *R, const double *Bb, double *D, double *Lo,
                              double *Up, hipStream_t s)
{
    hipLaunchKernelGGL(k_abd_to_btri, dim3(grid1((N + 1) * m * m, 256)), dim3(256), 0, s, m, N,
                       qa, Ba, S, R, Bb, D, Lo, Up);
    return hipGetLastError();
}

}  // namespace pf
