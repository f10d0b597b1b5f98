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
        if (threadIdx.x == 0) atomicMax(normA, dbits(a));
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const double a = block_max(mr[c], sh);
        const double b = block_max(mx[c], sh);
        const double d = block_max(mf[c], sh);
        if (threadIdx.x == 0 && c < nc) {
            atomicMax(norms + 3 * (c0 + c) + 0, dbits(a));
            atomicMax(norms + 3 * (c0 + c) + 1, dbits(b));
            atomicMax(norms + 3 * (c0 + c) + 2, dbits(d));
        }
    }
}

// The residual r = f - A x and the norms of eta on the matrix cores (FP64
// v_mfma_f64_16x16x4f64), for block sizes MB = 4, 8, 16, 32.  A wave takes
// a group of RG = max(16, MB) consecutive rows: the group's rows of A, over
// the window of RG + 2 MB columns its blocks touch (block columns of its
// first block row - 1 through its last + 1), are loaded once into registers
// as the A operands of RG/16 row tiles x (RG + 2 MB)/4 steps (K index of step
// s and lane group g: window column 4s + g), entries outside the three block
// diagonals zero; then every column tile of 16 right-hand sides is one chain
// of steps whose B operand is the x window, and r = f - acc in the result
// layout (lane (n, g): rows 4q + g of the tile, column n).  So A is read once
// per 64 right-hand sides (blockIdx.y), and a lane issues one x load per
// matrix-core step instead of one per multiply-add.  The BABD corner C (block
// row 0 against x[nb-1]) is a further chain in the group holding row 0.
// ||A||_inf (normA, first column chunk): per row the sum of |A| over its
// window entries and the corner, summed across the four lane groups.
template <int MB>
__global__ __launch_bounds__(256) void k_residual_mma(int kind, int64_t nb,
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
    typedef double v4 __attribute__((ext_vector_type(4)));
    constexpr int TI = MB > 16 ? MB / 16 : 1;   // row tiles per group
    constexpr int RG = 16 * TI;                 // rows per group
    constexpr int KS = (RG + 2 * MB) / 4;       // steps over the column window
    constexpr int KC = MB / 4;                  // steps of the corner chain
    constexpr int CT = 4;                       // column tiles per chunk
    constexpr int UJ = MB > 16 ? 1 : CT;        // their loop: unrolled below 32 x 32
    constexpr int SH = MB == 4 ? 2 : MB == 8 ? 3 : MB == 16 ? 4 : 5;
    constexpr int64_t MM = (int64_t)MB * MB;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int64_t N = (int64_t)MB * nb;
    const int64_t groups = (N + RG - 1) / RG;
    const int cb = blockIdx.y * (16 * CT);
    const bool wantA = normA != nullptr && blockIdx.y == 0;

    // A(i, j) of the block tridiagonal (kind 0) or bidiagonal (kind 1)
    // pattern, zero outside it and outside the matrix
    auto a_at = [&](int64_t i, int64_t j) -> double {
        if (i >= N || j < 0 || j >= N) return 0.0;
        const int64_t k = i >> SH, kc = j >> SH;
        const int64_t off = (i & (MB - 1)) + (j & (MB - 1)) * (int64_t)MB;
        if (kc == k) return D[k * MM + off];
        if (kc == k - 1) return Lo[(k - 1) * MM + off];
        if (kc == k + 1 && kind == 0) return Up[k * MM + off];
        return 0.0;
    };

    // per column of the chunk, this wave's running maxima of |r|, |x|, |f|
    // (entry (3J + t) 16 + n of its LDS row; only the wave itself touches it)
    __shared__ double sh[4][3 * CT * 16];
    __shared__ double sha[4];
    double ma = 0.0;
    for (int e = lane; e < 3 * CT * 16; e += 64) sh[wv][e] = 0.0;

    for (int64_t grp = (int64_t)blockIdx.x * 4 + wv; grp < groups;
         grp += (int64_t)gridDim.x * 4) {
        const int64_t row0 = grp * RG, w0 = row0 - MB;   // first row; first window column
        const bool corner = kind == 1 && row0 == 0;      // wave-uniform
        double a[TI][KS];
#pragma unroll
        for (int I = 0; I < TI; ++I)
#pragma unroll
            for (int st = 0; st < KS; ++st) a[I][st] = a_at(row0 + 16 * I + n, w0 + 4 * st + g);
        // the corner's A operand: C(16I + n, 4st + g) for rows of block row 0
        auto c_at = [&](int I, int st) -> double {
            const int i = 16 * I + n, j = 4 * st + g;
            return i < MB ? C[i + (int64_t)j * MB] : 0.0;
        };
        if (wantA) {
#pragma unroll
            for (int I = 0; I < TI; ++I) {
                double sa = 0.0;
#pragma unroll
                for (int st = 0; st < KS; ++st) sa += fabs(a[I][st]);
                if (corner)
#pragma unroll
                    for (int st = 0; st < KC; ++st) sa += fabs(c_at(I, st));
                sa += __shfl_xor(sa, 16, 64);
                sa += __shfl_xor(sa, 32, 64);
                ma = fmax(ma, sa);
            }
        }
#pragma unroll UJ
        for (int J = 0; J < CT; ++J) {
            const int c0 = cb + 16 * J;
            if (c0 >= nrhs) break;   // wave-uniform
            double mr = 0.0, mx = 0.0, mf = 0.0;
            const bool act = c0 + n < nrhs;
            const int64_t cc = act ? c0 + n : c0;   // an existing column (loads in bounds)
            double b[KS];
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                const int64_t j = w0 + 4 * st + g;
                b[st] = (act && j >= 0 && j < N) ? x[j + cc * ldx] : 0.0;
            }
            v4 acc[TI];
#pragma unroll
            for (int I = 0; I < TI; ++I) {
                acc[I] = v4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < KS; ++st)
                    acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I][st], b[st], acc[I], 0, 0, 0);
            }
            if (corner) {
#pragma unroll
                for (int st = 0; st < KC; ++st) {
                    const double bc = act ? x[(nb - 1) * MB + 4 * st + g + cc * ldx] : 0.0;
#pragma unroll
                    for (int I = 0; I < TI; ++I)
                        acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(c_at(I, st), bc, acc[I], 0, 0, 0);
                }
            }
            // the group's own rows of x are window steps MB/4 .. MB/4 + RG/4 - 1
#pragma unroll
            for (int st = MB / 4; st < MB / 4 + RG / 4; ++st) mx = fmax(mx, fabs(b[st]));
#pragma unroll
            for (int I = 0; I < TI; ++I)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t row = row0 + 16 * I + 4 * q + g;
                    if (act && row < N) {
                        const double fv = f[row + cc * ldf];
                        const double rv = fv - acc[I][q];
                        if (r) r[row + cc * ldr] = rv;
                        mr = fmax(mr, fabs(rv));
                        mf = fmax(mf, fabs(fv));
                    }
                }
            // column n's maxima over the four lane groups, into the wave's row
            double v[3] = {mr, mx, mf};
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                v[t] = fmax(v[t], __shfl_xor(v[t], 16, 64));
                v[t] = fmax(v[t], __shfl_xor(v[t], 32, 64));
                double &cell = sh[wv][(3 * J + t) * 16 + n];
                if (g == 0) cell = fmax(cell, v[t]);
            }
        }
    }
    // the workgroup's waves, then one atomic per column and norm
    if (wantA) {
        ma = wave_max(ma);
        if (lane == 0) sha[wv] = ma;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * CT * 16; e += blockDim.x) {
        const int J = e / 48, t = (e / 16) % 3, col = cb + 16 * J + (e & 15);
        if (col < nrhs) {
            const double v = fmax(fmax(sh[0][e], sh[1][e]), fmax(sh[2][e], sh[3][e]));
            atomicMax(norms + 3 * col + t, dbits(v));
        }
    }
    if (wantA && threadIdx.x == 0)
        atomicMax(normA, dbits(fmax(fmax(sha[0], sha[1]), fmax(sha[2], sha[3]))));
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
        auto mma = [&](auto mb) {
            constexpr int MB = decltype(mb)::value;
            constexpr int RG = MB > 16 ? MB : 16;
            const int64_t groups = (n + RG - 1) / RG;
            int64_t wg = (groups + 3) / 4;
            if (wg > 1024) wg = 1024;
            hipLaunchKernelGGL((k_residual_mma<MB>), dim3((unsigned)wg, (nrhs + 63) / 64), dim3(256),
                               0, s, kind, nb, D, Lo, Up, C, nrhs, f, ldf, x, ldx, r, ldr, norms,
                               normA);
            return hipGetLastError();
        };
        switch (m) {
        case 4: return mma(std::integral_constant<int, 4>{});
        case 8: return mma(std::integral_constant<int, 8>{});
        case 16: return mma(std::integral_constant<int, 16>{});
        default: return mma(std::integral_constant<int, 32>{});
        }
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

hipError_t launch_axpy(int64_t n, int32_t nrhs, const double *d, int64_t ldd, double *x,
                       int64_t ldx, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy, dim3(grid1(n, 256), nrhs), dim3(256), 0, s, n, d, ldd, x, ldx);
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
