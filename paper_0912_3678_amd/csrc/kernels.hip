// Partition-method kernels for gfx950 (CDNA4).
//
// Method (Amodio & Brugnano, Sec. 2): the block rows are split into p
// partitions separated by single separator block rows (eq. (parpart) for a
// block tridiagonal matrix, eq. (parpart1) for the bidiagonal-plus-corner
// form).  Each partition factors its local block M^(i) of eq. (Mi0) with the
// LU variant of eq. (parblock): a block Gaussian elimination down the
// partition that also carries the two fill-in spikes -- the left-separator
// column spike (paper z) and, for block tridiagonal matrices, the
// left-separator row spike (paper w) -- and ends with the partition's
// contributions alpha_1, alpha_2, beta, gamma to the reduced matrix of
// eq. (redmatr) / (redmatr1).
//
// GPU mapping.  A workgroup is one wave64.  A partition is owned by a group
// of M consecutive lanes (M = block size; 64/M partitions per wave) and lane
// i holds row i of every block the partition works on.  The pivot block is
// inverted by a row-distributed Gauss-Jordan elimination whose pivot search
// is a DPP reduction inside the group; operands that every lane needs in
// full go through the group's own, bank-padded slice of LDS.  A group never
// leaves its wave, so the only ordering needed between an LDS write and the
// reads of the other lanes is the in-order LDS pipe of the wave plus a
// compiler fence (wave_sync); no workgroup barrier is used.
//
// Memory discipline inside the chain loops: no memory operation sits under
// a branch (missing operands are read from a zero block, stores a lane must
// not make go to a dump buffer, the zero-pivot report is deferred), and the
// operands of the next block row are loaded before the current row's
// stores.  The compiler's wait counters then stay exact and a row never waits
// for the stores of the previous one (loads and stores share one in-order
// counter on this architecture).
//
// Factor storage: per block row g, row-major M x M blocks E (inverse of the
// eliminated pivot block D'), X = E A(g,g+1), Zh (left spike column) and R
// (left spike row) -- exactly the quantities the solve needs, laid out so the
// solve kernels load contiguous rows.
//
// Recurrences of one partition (global blocks g_1..g_n between the
// separators sL = g_1 - 1 and sR = g_n + 1), block tridiagonal case:
//   D'_1 = D[g_1],  Z'_1 = A(g_1, sL),  R_1 = A(sL, g_1)
//   for k = 1..n:
//     E_k = D'_k^{-1}                    (Gauss-Jordan, row partial pivoting)
//     X_k = E_k A(g_k, g_k+1),  Zh_k = E_k Z'_k
//     alpha_1 -= R_k Zh_k,      R_{k+1} = -R_k X_k
//     D'_{k+1} = D[g_k+1] - A(g_k+1, g_k) X_k,   Z'_{k+1} = -A(g_k+1, g_k) Zh_k
// At k = n the "next" quantities are the partition's contributions to the
// right separator: D'_{n+1} = D[sR] + alpha_2 (written as the reduced
// diagonal), Z'_{n+1} = beta, and R_{n+1} = gamma.
// Solve:  t_k = E_k (f_k - A(g_k, g_k-1) t_{k-1}),  g_sL -= sum R_k t_k,
//         g_sR -= A(sR, g_n) t_n;  then
//         x_k = t_k - Zh_k x_sL - X_k x_{k+1}  (x_{n+1} = x_sR).
// In the bidiagonal-plus-corner case A(g, g+1) = 0, so X = R = 0 and the
// back substitution is independent row by row (eq. (pups)).
#include "pf_internal.h"

#include <type_traits>

namespace pf {
namespace {

constexpr int WG = 64;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


__device__ __forceinline__ unsigned long long status_code(int level, int64_t block)
{
    return ((unsigned long long)level << 40) | (unsigned long long)block;
}

// ---- partition geometry ---------------------------------------------------
// Balanced rule: the non-separator blocks are spread as evenly as possible,
// the first (count mod p) partitions getting one block more.
struct Geo {
    int64_t start;   // first block of the partition
    int len;         // blocks in the partition
    int kmax;        // longest partition (uniform loop bound)
    bool valid, hasL, hasR;
};

template <int KIND>
__device__ __forceinline__ Geo geometry(int64_t nb, int64_t p, int64_t part)
{
    Geo g;
    const int64_t nint = (KIND == 0) ? nb - (p - 1) : nb - (p + 1);
    const int64_t q = nint / p, rem = nint % p;
    g.valid = part < p;
    const int64_t mn = part < rem ? part : rem;
    g.start = (KIND == 0 ? 0 : 1) + part * (q + 1) + mn;
    g.len = g.valid ? (int)(q + (part < rem ? 1 : 0)) : 0;
    g.kmax = (int)(q + (rem > 0 ? 1 : 0));
    if (KIND == 0) {
        g.hasL = g.valid && part > 0;
        g.hasR = g.valid && part < p - 1;
    } else {
        g.hasL = g.valid;
        g.hasR = g.valid;
    }
    return g;
}

// ---- register <-> memory helpers ------------------------------------------
// M contiguous doubles -> registers of type T
template <int M, typename T>
__device__ __forceinline__ void ld_vec(T (&v)[M], const double *__restrict__ p)
{
    if constexpr (M % 2 == 0) {
#pragma unroll
        for (int r = 0; r < M; r += 2) {
            const double2 w = *reinterpret_cast<const double2 *>(p + r);
            v[r] = (T)w.x;
            v[r + 1] = (T)w.y;
        }
    } else {
#pragma unroll
        for (int r = 0; r < M; ++r) v[r] = (T)p[r];
    }
}

template <int M, typename T>
__device__ __forceinline__ void add_vec(T (&v)[M], const double *__restrict__ p)
{
    T w[M];
    ld_vec<M, T>(w, p);
#pragma unroll
    for (int r = 0; r < M; ++r) v[r] += w[r];
}

// registers -> M contiguous T (16-byte stores where the size allows)
template <int M, typename T>
__device__ __forceinline__ void st_fac(T *__restrict__ p, const T (&v)[M])
{
    if constexpr (sizeof(T) == 8 && M % 2 == 0) {
#pragma unroll
        for (int r = 0; r < M; r += 2)
            *reinterpret_cast<double2 *>(p + r) = make_double2(v[r], v[r + 1]);
    } else if constexpr (sizeof(T) == 4 && M % 4 == 0) {
#pragma unroll
        for (int r = 0; r < M; r += 4)
            *reinterpret_cast<float4 *>(p + r) = make_float4(v[r], v[r + 1], v[r + 2], v[r + 3]);
    } else {
#pragma unroll
        for (int r = 0; r < M; ++r) p[r] = v[r];
    }
}

// M contiguous T (factor storage) -> registers (16-byte loads where possible)
template <int M, typename T>
__device__ __forceinline__ void ld_fac(T (&v)[M], const T *__restrict__ p)
{
    if constexpr (sizeof(T) == 8 && M % 2 == 0) {
#pragma unroll
        for (int r = 0; r < M; r += 2) {
            const double2 w = *reinterpret_cast<const double2 *>(p + r);
            v[r] = w.x;
            v[r + 1] = w.y;
        }
    } else if constexpr (sizeof(T) == 4 && M % 4 == 0) {
#pragma unroll
        for (int r = 0; r < M; r += 4) {
            const float4 w = *reinterpret_cast<const float4 *>(p + r);
            v[r] = w.x; v[r + 1] = w.y; v[r + 2] = w.z; v[r + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < M; ++r) v[r] = p[r];
    }
}

template <int M, typename T>
__device__ __forceinline__ void ld_row_d(T (&v)[M], const double *__restrict__ blk, int i)
{
#pragma unroll
    for (int l = 0; l < M; ++l) v[l] = (T)blk[i + l * M];
}

template <int M, typename T>
__device__ __forceinline__ void zero(T (&v)[M])
{
#pragma unroll
    for (int r = 0; r < M; ++r) v[r] = T(0);
}

template <int M, typename T>
__device__ __forceinline__ void mask(T (&v)[M], bool keep)
{
#pragma unroll
    for (int r = 0; r < M; ++r) v[r] = keep ? v[r] : T(0);
}

// column j of an M x M LDS matrix (column-major) <- v
template <int M, typename T>
__device__ __forceinline__ void lds_put_col(T *S, int j, const T (&v)[M])
{
#pragma unroll
    for (int r = 0; r < M; ++r) S[r + j * M] = v[r];
}

// o1 = S v1, o2 = S v2 with S an M x M column-major LDS matrix
template <int M, typename T>
__device__ __forceinline__ void lds_gemv2(const T *S, const T (&v1)[M], const T (&v2)[M],
                                          T (&o1)[M], T (&o2)[M])
{
    zero<M, T>(o1);
    zero<M, T>(o2);
#pragma unroll
    for (int l = 0; l < M; ++l) {
        T col[M];
#pragma unroll
        for (int r = 0; r < M; ++r) col[r] = S[r + l * M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
            o1[r] = fma(col[r], v1[l], o1[r]);
            o2[r] = fma(col[r], v2[l], o2[r]);
        }
    }
}

template <int M, typename T>
__device__ __forceinline__ void lds_gemv(const T *S, const T (&v)[M], T (&o)[M])
{
    zero<M, T>(o);
#pragma unroll
    for (int l = 0; l < M; ++l) {
#pragma unroll
        for (int r = 0; r < M; ++r) o[r] = fma(S[r + l * M], v[l], o[r]);
    }
}

// ---- LDS layout ---------------------------------------------------------------
// Rows of the small matrices a group keeps in LDS are padded by 16 bytes and
// the groups' regions start 16 bytes apart modulo 128, so the lanes of a group
// (one row each) and the groups of a wave (one region each) fall into
// different banks instead of all hitting the same one.
template <typename T> constexpr int kPad = 16 / (int)sizeof(T);
template <typename T> constexpr int kLine = 128 / (int)sizeof(T);
template <typename T> constexpr int group_stride(int elems)
{
    return ((elems + kLine<T> - 1) / kLine<T>) * kLine<T> + kPad<T>;
}

// ---- pivot search: group-wide max of a packed key with DPP ----------------
// A candidate's key is the high 32 bits of |v| (sign cleared) with the low 5
// bits replaced by 31 - row: an unsigned max over the group then picks the
// largest magnitude, compared to 15 (FP64) or 18 (FP32) mantissa bits, and
// among equal keys the first row.  Rows already used as pivots have key 0,
// below every candidate.  Each reduction stage is one max with a DPP operand.
template <int CTRL> __device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ unsigned pivot_key(double v, int row, bool used)
{
    const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(v) >> 32) & 0x7fffffffu;
    return used ? 0u : ((hi & ~31u) | (unsigned)(31 - row));
}
__device__ __forceinline__ unsigned pivot_key(float v, int row, bool used)
{
    const unsigned b = (unsigned)__float_as_int(v) & 0x7fffffffu;
    return used ? 0u : ((b & ~31u) | (unsigned)(31 - row));
}

// The M lanes of a group are an aligned run inside a row of 16 (M <= 16) or a
// half wave (M = 32), so these cross-lane moves never leave the group.
template <int M>
__device__ __forceinline__ int group_pivot(unsigned k)
{
    if constexpr (M >= 2) k = max(k, (unsigned)dpp_i<0xB1>((int)k));    // lane ^ 1
    if constexpr (M >= 4) k = max(k, (unsigned)dpp_i<0x4E>((int)k));    // lane ^ 2
    if constexpr (M >= 8) k = max(k, (unsigned)dpp_i<0x141>((int)k));   // half-row mirror
    if constexpr (M >= 16) k = max(k, (unsigned)dpp_i<0x140>((int)k));  // row mirror
    if constexpr (M >= 32) k = max(k, (unsigned)__shfl_xor((int)k, 16, 32));
    return 31 - (int)(k & 31u);
}

// reciprocal: hardware estimate refined by Newton steps (two in FP64, one in FP32)
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// ---- Gauss-Jordan inversion of the pivot block with row partial pivoting --
// Row-distributed and swap-free: lane i holds row i of D' in d (consumed) and
// starts with row i of the identity in e.  At step c the pivot is the row
// with the largest |D'(r,c)| among rows not yet used as pivots (ranked by
// pivot_key), found by a DPP max-reduction; the pivot lane's row [d | e] is read
// from the group's LDS, the pivot row is scaled by 1/pivot and column c is
// eliminated from every other row.  Rows never move: the lane chosen at step
// c ends with row c of D'^{-1} in e, and sigma (the return value) is c.
// Only the columns > c of d are still needed after step c.
template <int M, typename T>
__device__ __forceinline__ int gj_rows(T (&d)[M], T (&e)[M], int i, T *SP, bool &sing)
{
    constexpr int PR = 2 * M + kPad<T>;   // padded row stride of SP
#pragma unroll
    for (int l = 0; l < M; ++l) e[l] = (l == i) ? T(1) : T(0);
    bool used = false;
    int sigma = 0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const int pr = group_pivot<M>(pivot_key(d[c], i, used));
        T *row = SP + i * PR;
#pragma unroll
        for (int l = c; l < M; ++l) row[l] = d[l];
#pragma unroll
        for (int l = 0; l < M; ++l) row[M + l] = e[l];
        wave_sync();
        const T *prow = SP + pr * PR;
        T pd[M], pe[M];
#pragma unroll
        for (int l = c; l < M; ++l) pd[l] = prow[l];
#pragma unroll
        for (int l = 0; l < M; ++l) pe[l] = prow[M + l];
        const T pv = pd[c];
        sing = sing || (pv == T(0));
        const T inv = recip(pv);
        const bool isp = (i == pr);
        const T f = isp ? -inv : d[c] * inv;
        const T s = isp ? T(0) : T(1);
#pragma unroll
        for (int l = c + 1; l < M; ++l) d[l] = fma(-f, pd[l], s * d[l]);
#pragma unroll
        for (int l = 0; l < M; ++l) e[l] = fma(-f, pe[l], s * e[l]);
        used = used || isp;
        sigma = isp ? c : sigma;
        wave_sync();
    }
    return sigma;
}

// store row i of an M x M column-major FP64 block
template <int M, typename T>
__device__ __forceinline__ void st_row_d(double *__restrict__ blk, int i, const T (&v)[M])
{
#pragma unroll
    for (int l = 0; l < M; ++l) blk[i + l * M] = (double)v[l];
}

// ---------------------------------------------------------------------------
// Block tridiagonal factor: one level.  Lane i of a group holds row i of the
// running blocks D', Z', R and alpha_1.  ADD: the diagonal blocks are the sum
// of two arrays (the two neighbours' contributions of the level above).
template <int M, typename T, bool ADD>
__device__ __forceinline__ void btri_factor_body(const LevelArgs &a, int64_t pblock)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, i = tid % M;
    constexpr int RS = M + kPad<T>, PR = 2 * M + kPad<T>;
    constexpr int GS = group_stride<T>(M * PR + 2 * M * RS);
    __shared__ __align__(16) T lds[GPW * GS];
    T *SP = lds + grp * GS;   // Gauss-Jordan pivot rows (M x PR)
    T *SU = SP + M * PR;      // A(g,g+1)^T, then the rows of X (M x RS)
    T *SZ = SU + M * RS;      // Z'^T, then the rows of Zh (M x RS)

    const int64_t nb = a.nb;
    const int64_t part = pblock * GPW + grp;
    const Geo G = geometry<0>(nb, a.p, part);
    T *E = (T *)a.E, *R = (T *)a.R, *Zs = (T *)a.Z, *Xs = (T *)a.X;
    T *dump = (T *)a.dump + tid * M;

    T d[M], z[M], rr[M], a1[M];
    zero<M, T>(d); zero<M, T>(z); zero<M, T>(rr); zero<M, T>(a1);
    if (G.valid) {
        ld_row_d<M, T>(d, a.D + G.start * MM, i);
        if constexpr (ADD) {
            T w[M];
            ld_row_d<M, T>(w, a.Dadd + G.start * MM, i);
#pragma unroll
            for (int l = 0; l < M; ++l) d[l] += w[l];
        }
    }
    if (G.hasL) {
        ld_row_d<M, T>(z, a.Lo + (G.start - 1) * MM, i);   // A(g_1, sL)
        ld_row_d<M, T>(rr, a.Up + (G.start - 1) * MM, i);  // A(sL, g_1)
    }
    unsigned long long bad = ~0ull;

    // Operands of block row g that do not depend on the chain: column i of
    // A(g,g+1), row i of A(g+1,g) and of D[g+1].  They are loaded one row
    // ahead (before the stores of the current row), and from the zero block
    // when they do not exist.
    auto load_next = [&](int64_t g, bool ok, T (&upc)[M], T (&lor)[M], T (&dn)[M]) {
        ld_vec<M, T>(upc, (ok ? a.Up + g * MM : a.zero) + i * M);
        ld_row_d<M, T>(lor, ok ? a.Lo + g * MM : a.zero, i);
        ld_row_d<M, T>(dn, ok ? a.D + (g + 1) * MM : a.zero, i);
        if constexpr (ADD) {
            T w[M];
            ld_row_d<M, T>(w, ok ? a.Dadd + (g + 1) * MM : a.zero, i);
#pragma unroll
            for (int l = 0; l < M; ++l) dn[l] += w[l];
        }
    };
    T upc[M], lor[M], dn[M];
    load_next(G.start, G.len > 0 && G.start + 1 < nb, upc, lor, dn);

    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        T upn[M], lon[M], dnn[M];
        load_next(g + 1, k + 1 < G.len && g + 2 < nb, upn, lon, dnn);

        T e[M];
        bool sing = false;
        const int sig = gj_rows<M, T>(d, e, i, SP, sing);
        const unsigned long long code = status_code(a.level, g);
        bad = (sing && code < bad) ? code : bad;
        st_fac<M, T>(E + g * MM + sig * M, e);             // row sig of E_k
        st_fac<M, T>(G.hasL ? R + g * MM + i * M : dump, rr);   // row i of R_k
#pragma unroll
        for (int l = 0; l < M; ++l) {
            SU[i * RS + l] = upc[l];                       // row i of A(g,g+1)^T
            SZ[l * RS + i] = z[l];                         // column i of Z'^T
        }
        wave_sync();
        T x[M], zh[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {                      // row sig of X_k and Zh_k
            T sx = T(0), sz = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                sx = fma(e[l], SU[c * RS + l], sx);
                sz = fma(e[l], SZ[c * RS + l], sz);
            }
            x[c] = sx;
            zh[c] = sz;
        }
        st_fac<M, T>(Xs + g * MM + sig * M, x);
        st_fac<M, T>(Zs + g * MM + sig * M, zh);
        wave_sync();
#pragma unroll
        for (int c = 0; c < M; ++c) {
            SU[sig * RS + c] = x[c];
            SZ[sig * RS + c] = zh[c];
        }
        wave_sync();
        T rn[M], t1[M], dl[M], zl[M];
        zero<M, T>(rn); zero<M, T>(t1); zero<M, T>(dl); zero<M, T>(zl);
#pragma unroll
        for (int l = 0; l < M; ++l) {                      // R_k X_k, R_k Zh_k, Lo X_k, Lo Zh_k
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const T xv = SU[l * RS + c], zv = SZ[l * RS + c];
                rn[c] = fma(rr[l], xv, rn[c]);
                t1[c] = fma(rr[l], zv, t1[c]);
                dl[c] = fma(lor[l], xv, dl[c]);
                zl[c] = fma(lor[l], zv, zl[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            a1[c] -= t1[c];
            rr[c] = -rn[c];
            d[c] = dn[c] - dl[c];
            z[c] = -zl[c];
            upc[c] = upn[c];
            lor[c] = lon[c];
            dn[c] = dnn[c];
        }
        wave_sync();
    }
    if (bad != ~0ull) atomicMin(a.status, bad);
    // contributions to the reduced matrix (eq. (redmatr)); separator j sits
    // between partitions j and j+1
    if (G.hasR) {
        st_row_d<M, T>(a.nD + part * MM, i, d);                    // D[sR] + alpha_2
        if (G.hasL) st_row_d<M, T>(a.nLo + (part - 1) * MM, i, z); // beta
    }
    if (G.hasL) {
        st_row_d<M, T>(a.nDadd + (part - 1) * MM, i, a1);          // alpha_1
        if (G.hasR) st_row_d<M, T>(a.nUp + (part - 1) * MM, i, rr); // gamma
    }
}

// ---------------------------------------------------------------------------
// Bidiagonal-plus-corner factor: one level.  Separators s_0 = 0 < s_1 < ... <
// s_p = nb-1; partition `part` lies between s_part and s_{part+1}.  The
// reduced matrix (eq. (redmatr1) with gamma = 0) has the same form:
// diagonal D[s_i], sub-diagonal beta, corner unchanged.
template <int M, typename T>
__device__ __forceinline__ void babd_factor_body(const LevelArgs &a, int64_t pblock)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, i = tid % M;
    constexpr int RS = M + kPad<T>, PR = 2 * M + kPad<T>;
    constexpr int GS = group_stride<T>(M * PR + M * RS);
    __shared__ __align__(16) T lds[GPW * GS];
    T *SP = lds + grp * GS;   // Gauss-Jordan pivot rows
    T *SZ = SP + M * PR;      // Z'^T, then the rows of Zh

    const int64_t part = pblock * GPW + grp;
    const Geo G = geometry<1>(a.nb, a.p, part);
    T *E = (T *)a.E, *Zs = (T *)a.Z;

    T z[M];
    zero<M, T>(z);
    if (G.valid) ld_row_d<M, T>(z, a.Lo + (G.start - 1) * MM, i);   // A(g_1, sL)
    unsigned long long bad = ~0ull;

    // rows i of D[g] and A(g+1,g), loaded one block row ahead
    T dc[M], lc[M];
    ld_row_d<M, T>(dc, G.len > 0 ? a.D + G.start * MM : a.zero, i);
    ld_row_d<M, T>(lc, G.len > 0 ? a.Lo + G.start * MM : a.zero, i);
    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        const bool more = k + 1 < G.len;
        T d[M], lor[M];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            d[l] = dc[l];
            lor[l] = lc[l];
        }
        ld_row_d<M, T>(dc, more ? a.D + (g + 1) * MM : a.zero, i);
        ld_row_d<M, T>(lc, more ? a.Lo + (g + 1) * MM : a.zero, i);
        T e[M];
        bool sing = false;
        const int sig = gj_rows<M, T>(d, e, i, SP, sing);
        const unsigned long long code = status_code(a.level, g);
        bad = (sing && code < bad) ? code : bad;
        st_fac<M, T>(E + g * MM + sig * M, e);
#pragma unroll
        for (int l = 0; l < M; ++l) SZ[l * RS + i] = z[l];   // column i of Z'^T
        wave_sync();
        T zh[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T s = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) s = fma(e[l], SZ[c * RS + l], s);
            zh[c] = s;
        }
        st_fac<M, T>(Zs + g * MM + sig * M, zh);
        wave_sync();
#pragma unroll
        for (int c = 0; c < M; ++c) SZ[sig * RS + c] = zh[c];
        wave_sync();
        T zl[M];
        zero<M, T>(zl);
#pragma unroll
        for (int l = 0; l < M; ++l)
#pragma unroll
            for (int c = 0; c < M; ++c) zl[c] = fma(lor[l], SZ[l * RS + c], zl[c]);
#pragma unroll
        for (int c = 0; c < M; ++c) z[c] = -zl[c];
        wave_sync();
    }
    if (bad != ~0ull) atomicMin(a.status, bad);
    if (G.valid) {
        const int64_t sR = G.start + G.len;
        st_row_d<M, T>(a.nLo + part * MM, i, z);                     // beta
        const double *ds = a.D + sR * MM + i * M;                    // copy column i
        double *od = a.nD + (part + 1) * MM + i * M;
#pragma unroll
        for (int r = 0; r < M; ++r) od[r] = ds[r];
        if (part == 0) {
#pragma unroll
            for (int r = 0; r < M; ++r) {
                a.nD[i * M + r] = a.D[i * M + r];
                a.nC[i * M + r] = a.C[i * M + r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Tile mapping: one partition per M*M lanes (M = 2, 4, 8; 64/(M*M)
// partitions per wave).  Lane (r, c) of a partition holds entry (r, c) of
// every block of its chain, column c occupying M consecutive lanes.  The
// per-row work is spread over M times more lanes than in the row mapping,
// which cuts the latency of a chain row several times over: this mapping is
// for levels with few partitions (the reduced levels), where latency, not
// bandwidth, bounds a level.
//
// The pivot block is inverted in place by Gauss-Jordan exchange steps: step
// j exchanges unknown j with the equation of pivot row p_j (the largest
// |entry| of column j among the rows not yet used, as ranked by pivot_key).
// With b the running tableau and v = b(p_j, j):
//   b(p_j, j) <- 1/v,  b(p_j, l) <- b(p_j, l)/v,  b(i, j) <- -b(i, j)/v,
//   b(i, l) <- b(i, l) - b(i, j) b(p_j, l)/v          (i != p_j, l != j).
// After the M steps b(r, c) is entry (sigma(r), p_c) of the inverse, sigma(r)
// being the step at which row r was the pivot.  The pivot search of step
// j+1 is a DPP reduction inside column group j+1 right after step j's
// update, so each step costs one LDS round trip.

// pivot row of column j: reduce over column group j, then broadcast it to
// the partition's lanes
template <int M, typename T>
__device__ __forceinline__ int tile_pivot(T b, bool used, int r, int j)
{
    constexpr int LP = M * M;
    const int idx = group_pivot<M>(pivot_key(b, r, used));
    if constexpr (LP == WG) return __builtin_amdgcn_readlane(idx, j * M);
    else return __shfl(idx, (int)((threadIdx.x / LP) * LP) + j * M, WG);
}

// In-place Gauss-Jordan of the tableau b = D'(r, c); returns sigma(r) and
// p_c through the references.
template <int M, typename T>
__device__ __forceinline__ void tile_invert(T &b, int r, int c, T *S, int &sigma, int &pc,
                                            bool &sing)
{
    constexpr int RS = M + kPad<T>;
    bool used = false;
    int pr = tile_pivot<M, T>(b, used, r, 0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        S[r * RS + c] = b;
        wave_sync();
        const T prow = S[pr * RS + c], mcol = S[r * RS + j], pv = S[pr * RS + j];
        sing = sing || (pv == T(0));
        const T inv = recip(pv);
        const bool isr = (r == pr), isc = (c == j);
        const T upd = fma(-(mcol * inv), prow, b);
        b = isr ? (isc ? inv : prow * inv) : (isc ? -mcol * inv : upd);
        used = used || isr;
        sigma = isr ? j : sigma;
        pc = isc ? pr : pc;
        wave_sync();
        if (j + 1 < M) pr = tile_pivot<M, T>(b, used, r, j + 1);
    }
}

// M entries of an LDS row (16-byte reads; rows are 16-byte aligned)
template <int M, typename T>
__device__ __forceinline__ void lds_row(T (&v)[M], const T *p)
{
    if constexpr (sizeof(T) == 8 && M % 2 == 0) {
#pragma unroll
        for (int l = 0; l < M; l += 2) {
            const double2 w = *reinterpret_cast<const double2 *>(p + l);
            v[l] = w.x;
            v[l + 1] = w.y;
        }
    } else if constexpr (sizeof(T) == 4 && M % 4 == 0) {
#pragma unroll
        for (int l = 0; l < M; l += 4) {
            const float4 w = *reinterpret_cast<const float4 *>(p + l);
            v[l] = w.x; v[l + 1] = w.y; v[l + 2] = w.z; v[l + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int l = 0; l < M; ++l) v[l] = p[l];
    }
}

template <int M, typename T>
__device__ __forceinline__ T dot(const T (&u)[M], const T (&v)[M])
{
    T s = T(0);
#pragma unroll
    for (int l = 0; l < M; ++l) s = fma(u[l], v[l], s);
    return s;
}

// Block tridiagonal factor, tile mapping (same recurrences, storage and
// outputs as btri_factor_body).  RHS: the forward sweep of a solve runs in
// the same pass (factor-and-solve, the F solve of Sec. 2 next to the
// factorization): lane (r, c) also carries entry r of right-hand-side column
// c (c < nrhs <= M) of f' and t, and the level's t and reduced right-hand
// side are written as by fwd_body.
template <int M, typename T, bool ADD, bool RHS>
__device__ __forceinline__ void btri_factor_tile_body(const LevelArgs &a, const SolveArgs &sv,
                                                      int64_t pblock)
{
    constexpr int LP = M * M, PPW = WG / LP;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / LP, t = tid % LP;
    const int r = t % M, c = t / M;
    constexpr int RS = M + kPad<T>;
    constexpr int NS = RHS ? 5 : 4;
    constexpr int GS = group_stride<T>(NS * M * RS);
    __shared__ __align__(16) T lds[PPW * GS];
    T *S0 = lds + grp * GS;   // tableau; then E by rows; then R by rows
    T *S1 = S0 + M * RS;      // Z' by columns; then X by columns
    T *S2 = S1 + M * RS;      // A(g+1,g) by rows
    T *S3 = S2 + M * RS;      // Zh by columns
    T *S4 = S3 + M * RS;      // (RHS) f' by columns; then t by columns

    const int64_t nb = a.nb;
    const int64_t part = pblock * PPW + grp;
    const Geo G = geometry<0>(nb, a.p, part);
    T *E = (T *)a.E, *R = (T *)a.R, *Zs = (T *)a.Z, *Xs = (T *)a.X;
    T *dump = (T *)a.dump + tid;
    const int cm = r + c * M;   // column-major offset of (r, c)
    const int rm = r * M + c;   // row-major offset
    // right-hand-side column of this lane (RHS), clamped to an existing one
    const bool act = RHS && c < sv.nrhs;
    const int64_t fo = (int64_t)r + (int64_t)(act ? c : 0) * sv.ldf;
    const int64_t yo = (int64_t)r + (int64_t)(act ? c : 0) * sv.ldy;
    double *ydump = (double *)a.dump + WG + tid;

    T d = T(0), z = T(0), rr = T(0), a1 = T(0), fp = T(0), gl = T(0);
    if (G.valid) {
        double v = a.D[G.start * MM + cm];
        if constexpr (ADD) v += a.Dadd[G.start * MM + cm];
        d = (T)v;
        if constexpr (RHS) {
            double w = act ? sv.F[G.start * M + fo] : 0.0;
            if constexpr (ADD) w += act ? sv.Fadd[G.start * M + fo] : 0.0;
            fp = (T)w;
        }
    }
    if (G.hasL) {
        z = (T)a.Lo[(G.start - 1) * MM + cm];    // A(g_1, sL)
        rr = (T)a.Up[(G.start - 1) * MM + cm];   // A(sL, g_1)
    }
    unsigned long long bad = ~0ull;

    // column c of A(g,g+1), entry (r,c) of A(g+1,g), of D[g+1] and (RHS) of
    // f[g+1], one block row ahead, from the zero block when they do not
    // exist; the two addends of a sum stay apart until the row that uses them
    auto load_next = [&](int64_t g, bool ok, T (&upc)[M], T &lo, double &dn, double &da,
                         double &fn, double &fa) {
        ld_vec<M, T>(upc, (ok ? a.Up + g * MM : a.zero) + c * M);
        lo = (T)*((ok ? a.Lo + g * MM : a.zero) + cm);
        dn = *((ok ? a.D + (g + 1) * MM : a.zero) + cm);
        if constexpr (ADD) da = *((ok ? a.Dadd + (g + 1) * MM : a.zero) + cm);
        if constexpr (RHS) {
            fn = *((ok && act) ? sv.F + (g + 1) * M + fo : a.zero);
            if constexpr (ADD) fa = *((ok && act) ? sv.Fadd + (g + 1) * M + fo : a.zero);
        }
    };
    T upc[M], lo;
    double dn, da = 0.0, fn = 0.0, fa = 0.0;
    load_next(G.start, G.len > 0 && G.start + 1 < nb, upc, lo, dn, da, fn, fa);

    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        T upn[M], lon;
        double dnn, dan = 0.0, fnn = 0.0, fan = 0.0;
        load_next(g + 1, k + 1 < G.len && g + 2 < nb, upn, lon, dnn, dan, fnn, fan);

        T b = d;
        int sigma = 0, pc = 0;
        bool sing = false;
        tile_invert<M, T>(b, r, c, S0, sigma, pc, sing);
        const unsigned long long code = status_code(a.level, g);
        bad = (sing && code < bad) ? code : bad;

        S0[sigma * RS + pc] = b;   // E_k by (logical) rows
        S1[c * RS + r] = z;        // Z'_k by columns
        S2[r * RS + c] = lo;       // A(g+1,g) by rows
        if constexpr (RHS) S4[c * RS + r] = fp;   // f'_k by columns
        wave_sync();
        T er[M], zc[M], lr[M];
        lds_row<M, T>(er, S0 + r * RS);
        lds_row<M, T>(zc, S1 + c * RS);
        lds_row<M, T>(lr, S2 + r * RS);
        const T x = dot<M, T>(er, upc), zh = dot<M, T>(er, zc);
        T tk = T(0);
        if constexpr (RHS) {
            T fc[M];
            lds_row<M, T>(fc, S4 + c * RS);
            tk = dot<M, T>(er, fc);                              // t_k = E_k f'_k
            *(act ? sv.Y + g * M + yo : ydump) = (double)tk;
        }
        E[g * MM + sigma * M + pc] = b;
        *(G.hasL ? R + g * MM + rm : dump) = rr;
        Xs[g * MM + rm] = x;
        Zs[g * MM + rm] = zh;
        wave_sync();
        S0[r * RS + c] = rr;       // R_k by rows
        S1[c * RS + r] = x;        // X_k by columns
        S3[c * RS + r] = zh;       // Zh_k by columns
        if constexpr (RHS) S4[c * RS + r] = tk;   // t_k by columns
        wave_sync();
        T rw[M], xc[M], hc[M];
        lds_row<M, T>(rw, S0 + r * RS);
        lds_row<M, T>(xc, S1 + c * RS);
        lds_row<M, T>(hc, S3 + c * RS);
        a1 -= dot<M, T>(rw, hc);
        rr = -dot<M, T>(rw, xc);
        d = (T)(ADD ? dn + da : dn) - dot<M, T>(lr, xc);
        z = -dot<M, T>(lr, hc);
        if constexpr (RHS) {
            T tc[M];
            lds_row<M, T>(tc, S4 + c * RS);
            gl -= dot<M, T>(rw, tc);                             // g_sL -= R_k t_k
            fp = (T)(ADD ? fn + fa : fn) - dot<M, T>(lr, tc);    // f'_{k+1}
        }
#pragma unroll
        for (int l = 0; l < M; ++l) upc[l] = upn[l];
        lo = lon;
        dn = dnn;
        da = dan;
        fn = fnn;
        fa = fan;
        wave_sync();
    }
    if (bad != ~0ull) atomicMin(a.status, bad);
    if (G.hasR) {
        a.nD[part * MM + cm] = (double)d;                       // D[sR] + alpha_2
        if (G.hasL) a.nLo[(part - 1) * MM + cm] = (double)z;    // beta
    }
    if (G.hasL) {
        a.nDadd[(part - 1) * MM + cm] = (double)a1;             // alpha_1
        if (G.hasR) a.nUp[(part - 1) * MM + cm] = (double)rr;   // gamma
    }
    if constexpr (RHS) {
        if (act) {
            const int64_t no = (int64_t)r + (int64_t)c * sv.ldn;
            if (G.hasR) sv.nF[part * M + no] = (double)fp;          // f[sR] - A(sR,g_n) t_n
            if (G.hasL) sv.nFadd[(part - 1) * M + no] = (double)gl; // - sum R_k t_k
        }
    }
}

// Bidiagonal-plus-corner factor, tile mapping (same outputs as
// babd_factor_body).  D' = D here, so the inversion of the next block row
// does not wait for the chain.  RHS as in btri_factor_tile_body.
template <int M, typename T, bool RHS>
__device__ __forceinline__ void babd_factor_tile_body(const LevelArgs &a, const SolveArgs &sv,
                                                      int64_t pblock)
{
    constexpr int LP = M * M, PPW = WG / LP;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / LP, t = tid % LP;
    const int r = t % M, c = t / M;
    constexpr int RS = M + kPad<T>;
    constexpr int NS = RHS ? 5 : 4;
    constexpr int GS = group_stride<T>(NS * M * RS);
    __shared__ __align__(16) T lds[PPW * GS];
    T *S0 = lds + grp * GS;   // tableau; then E by rows
    T *S1 = S0 + M * RS;      // Z' by columns
    T *S2 = S1 + M * RS;      // A(g+1,g) by rows
    T *S3 = S2 + M * RS;      // Zh by columns
    T *S4 = S3 + M * RS;      // (RHS) f' by columns; then t by columns

    const int64_t part = pblock * PPW + grp;
    const Geo G = geometry<1>(a.nb, a.p, part);
    T *E = (T *)a.E, *Zs = (T *)a.Z;
    const int cm = r + c * M, rm = r * M + c;
    const bool act = RHS && c < sv.nrhs;
    const int64_t fo = (int64_t)r + (int64_t)(act ? c : 0) * sv.ldf;
    const int64_t yo = (int64_t)r + (int64_t)(act ? c : 0) * sv.ldy;
    double *ydump = (double *)a.dump + WG + tid;

    T z = G.valid ? (T)a.Lo[(G.start - 1) * MM + cm] : T(0);   // A(g_1, sL)
    T fp = T(0);
    if constexpr (RHS) fp = (G.valid && act) ? (T)sv.F[G.start * M + fo] : T(0);
    unsigned long long bad = ~0ull;
    T dc = (T)*((G.len > 0 ? a.D + G.start * MM : a.zero) + cm);
    T lc = (T)*((G.len > 0 ? a.Lo + G.start * MM : a.zero) + cm);
    double fc = 0.0;
    if constexpr (RHS) fc = *((G.len > 0 && act) ? sv.F + (G.start + 1) * M + fo : a.zero);
    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        const bool more = k + 1 < G.len;
        T b = dc;
        const T lo = lc;
        const double fn = fc;
        dc = (T)*((more ? a.D + (g + 1) * MM : a.zero) + cm);
        lc = (T)*((more ? a.Lo + (g + 1) * MM : a.zero) + cm);
        if constexpr (RHS) fc = *((more && act) ? sv.F + (g + 2) * M + fo : a.zero);

        int sigma = 0, pc = 0;
        bool sing = false;
        tile_invert<M, T>(b, r, c, S0, sigma, pc, sing);
        const unsigned long long code = status_code(a.level, g);
        bad = (sing && code < bad) ? code : bad;

        S0[sigma * RS + pc] = b;
        S1[c * RS + r] = z;
        S2[r * RS + c] = lo;
        if constexpr (RHS) S4[c * RS + r] = fp;
        wave_sync();
        T er[M], zc[M], lr[M];
        lds_row<M, T>(er, S0 + r * RS);
        lds_row<M, T>(zc, S1 + c * RS);
        lds_row<M, T>(lr, S2 + r * RS);
        const T zh = dot<M, T>(er, zc);
        T tk = T(0);
        if constexpr (RHS) {
            T fv[M];
            lds_row<M, T>(fv, S4 + c * RS);
            tk = dot<M, T>(er, fv);
            *(act ? sv.Y + g * M + yo : ydump) = (double)tk;
        }
        E[g * MM + sigma * M + pc] = b;
        Zs[g * MM + rm] = zh;
        S3[c * RS + r] = zh;
        if constexpr (RHS) S4[c * RS + r] = tk;
        wave_sync();
        T hc[M];
        lds_row<M, T>(hc, S3 + c * RS);
        z = -dot<M, T>(lr, hc);
        if constexpr (RHS) {
            T tc[M];
            lds_row<M, T>(tc, S4 + c * RS);
            fp = (T)fn - dot<M, T>(lr, tc);
        }
        wave_sync();
    }
    if (bad != ~0ull) atomicMin(a.status, bad);
    if (G.valid) {
        const int64_t sR = G.start + G.len;
        a.nLo[part * MM + cm] = (double)z;                         // beta
        a.nD[(part + 1) * MM + cm] = a.D[sR * MM + cm];
        if (part == 0) {
            a.nD[cm] = a.D[cm];
            a.nC[cm] = a.C[cm];
        }
        if constexpr (RHS) {
            if (act) {
                const int64_t no = (int64_t)r + (int64_t)c * sv.ldn;
                sv.nF[(part + 1) * M + no] = (double)fp;
                if (part == 0) sv.nF[no] = sv.F[fo];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Forward sweep of a solve (the F solve): t_k and the reduced right-hand side.
// Lane i owns row i of KC right-hand-side columns.  ADD: the right-hand side
// is the sum of two arrays (reduced levels of block tridiagonal matrices).
template <int KIND, int M, int KC, typename T, bool ADD>
__device__ __forceinline__ void fwd_body(const SolveArgs &a, int64_t pblock, int cblock)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, i = tid % M;
    constexpr int CS = M + kPad<T>;                   // padded column stride
    constexpr int GS = group_stride<T>(KC * CS);
    __shared__ __align__(16) T lds[GPW * GS];
    T *SV = lds + grp * GS;                           // M x KC block vector, by columns
    const int64_t part = pblock * GPW + grp;
    const Geo G = geometry<KIND>(a.nb, a.p, part);
    const int c0 = cblock * KC;
    const int kc = (a.nrhs - c0) < KC ? (a.nrhs - c0) : KC;
    const T *E = (const T *)a.E, *R = (const T *)a.R;
    double *dump = a.dump + tid;

    int64_t col[KC];   // column offsets, clamped to existing columns
#pragma unroll
    for (int c = 0; c < KC; ++c) col[c] = (int64_t)(c0 + (c < kc ? c : kc - 1));

    T fp[KC], gl[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
        fp[c] = T(0);
        gl[c] = T(0);
        if (G.valid) {
            double v = a.F[G.start * M + i + col[c] * a.ldf];
            if constexpr (ADD) v += a.Fadd[G.start * M + i + col[c] * a.ldf];
            fp[c] = (T)v;
        }
    }
    // Row i of E_g, R_g and A(g+1,g) and row i of the next right-hand side,
    // loaded one block row ahead (before the current row's stores); missing
    // operands come from the zero block.
    const T *zt = (const T *)a.zero + i * M;
    // (the right-hand side stays in FP64 and its two addends apart until the
    // row that uses them: converting or summing early would wait for this
    // row's own prefetch)
    auto load_row = [&](int64_t g, bool ok, T (&er)[M], T (&rr)[M], T (&lr)[M],
                        double (&fn)[KC], double (&fa)[KC]) {
        const bool nx = ok && (g + 1 < a.nb);
        ld_fac<M, T>(er, ok ? E + g * MM + i * M : zt);
        if constexpr (KIND == 0) ld_fac<M, T>(rr, (ok && G.hasL) ? R + g * MM + i * M : zt);
        ld_row_d<M, T>(lr, nx ? a.Lo + g * MM : a.zero, i);
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            const int64_t o = (g + 1) * M + i + col[c] * a.ldf;
            fn[c] = *(nx ? a.F + o : a.zero);
            if constexpr (ADD) fa[c] = *(nx ? a.Fadd + o : a.zero);
        }
    };
    T ec[M], rc[M], lc[M];
    double fc[KC], fca[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) fca[c] = 0.0;
    load_row(G.start, G.len > 0, ec, rc, lc, fc, fca);
    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        T er[M], lr[M], rr[M];
        double fn[KC], fna[KC];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            er[l] = ec[l];
            lr[l] = lc[l];
            if constexpr (KIND == 0) rr[l] = rc[l];
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            fn[c] = fc[c];
            fna[c] = fca[c];
        }
        load_row(g + 1, k + 1 < G.len, ec, rc, lc, fc, fca);
#pragma unroll
        for (int c = 0; c < KC; ++c) SV[i + c * CS] = fp[c];
        wave_sync();
        T t[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T s = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) s = fma(er[l], SV[l + c * CS], s);
            t[c] = s;
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            double *dst = (c < kc) ? a.Y + g * M + i + col[c] * a.ldy : dump;
            *dst = (double)t[c];
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) SV[i + c * CS] = t[c];
        wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T sl = T(0), sr = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                const T tv = SV[l + c * CS];
                sl = fma(lr[l], tv, sl);
                if constexpr (KIND == 0) sr = fma(rr[l], tv, sr);
            }
            fp[c] = (T)(ADD ? fn[c] + fna[c] : fn[c]) - sl;
            if constexpr (KIND == 0) gl[c] -= sr;
        }
        wave_sync();
    }
#pragma unroll
    for (int c = 0; c < KC; ++c) {
        if (c >= kc) continue;
        const int64_t cn = col[c] * a.ldn;
        if (KIND == 0) {
            if (G.hasR) a.nF[part * M + i + cn] = (double)fp[c];
            if (G.hasL) a.nFadd[(part - 1) * M + i + cn] = (double)gl[c];
        } else if (G.valid) {
            a.nF[(part + 1) * M + i + cn] = (double)fp[c];
            if (part == 0) a.nF[i + cn] = a.F[i + col[c] * a.ldf];
        }
    }
}

// ---------------------------------------------------------------------------
// Back substitution (the G solve / the parallel updates of eq. (pups)).
template <int KIND, int M, int KC, typename T>
__device__ __forceinline__ void bwd_body(const SolveArgs &a, int64_t pblock, int cblock)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, i = tid % M;
    constexpr int CS = M + kPad<T>;                   // padded column stride
    constexpr int GS = group_stride<T>(2 * KC * CS);
    __shared__ __align__(16) T lds[GPW * GS];
    T *SV = lds + grp * GS;                           // x of the row below (M x KC)
    T *SL = SV + KC * CS;                             // x at the left separator
    const int64_t part = pblock * GPW + grp;
    const Geo G = geometry<KIND>(a.nb, a.p, part);
    const int c0 = cblock * KC;
    const int kc = (a.nrhs - c0) < KC ? (a.nrhs - c0) : KC;
    const T *Zs = (const T *)a.Z, *Xs = (const T *)a.X;
    double *dump = a.dump + tid;
    const int64_t sR = G.start + G.len;
    // reduced-solution indices of the two separators
    const int64_t jl = (KIND == 0) ? part - 1 : part;
    const int64_t jr = (KIND == 0) ? part : part + 1;

    int64_t col[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) col[c] = (int64_t)(c0 + (c < kc ? c : kc - 1));

#pragma unroll
    for (int c = 0; c < KC; ++c) {
        T xl = T(0), xr = T(0);
        if (c < kc) {
            const int64_t cn = col[c] * a.ldn;
            if (G.hasL) xl = (T)a.Xsep[jl * M + i + cn];
            if (G.hasR) {
                const double v = a.Xsep[jr * M + i + cn];
                xr = (T)v;
                a.Y[sR * M + i + col[c] * a.ldy] = v;
            }
            if (KIND == 1 && G.valid && part == 0) a.Y[i + col[c] * a.ldy] = a.Xsep[i + cn];
        }
        SL[i + c * CS] = xl;
        SV[i + c * CS] = xr;
    }
    wave_sync();
    for (int k = G.len - 1; k >= 0; --k) {
        const int64_t g = G.start + k;
        T zr[M], xrw[M], t[KC];
        ld_fac<M, T>(zr, Zs + g * MM + i * M);
        if constexpr (KIND == 0) ld_fac<M, T>(xrw, Xs + g * MM + i * M);
#pragma unroll
        for (int c = 0; c < KC; ++c) t[c] = (T)a.Y[g * M + i + col[c] * a.ldy];
        T xk[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T s = t[c];
#pragma unroll
            for (int l = 0; l < M; ++l) {
                s = fma(-zr[l], SL[l + c * CS], s);
                if constexpr (KIND == 0) s = fma(-xrw[l], SV[l + c * CS], s);
            }
            xk[c] = s;
        }
        if constexpr (KIND == 0) wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            double *dst = (c < kc) ? a.Y + g * M + i + col[c] * a.ldy : dump;
            *dst = (double)xk[c];
            if constexpr (KIND == 0) SV[i + c * CS] = xk[c];
        }
        if constexpr (KIND == 0) wave_sync();
    }
}

// ---- kernels: one system (the grid covers its partitions) and batched (a
// table of per-system arguments and a work list whose entry w says: system
// table[w.x], partition block w.y, right-hand-side block w.z) -----------------
template <int M, typename T, bool ADD>
__global__ __launch_bounds__(WG) void k_btri_factor(LevelArgs a)
{
    btri_factor_body<M, T, ADD>(a, blockIdx.x);
}
template <int M, typename T, bool ADD>
__global__ __launch_bounds__(WG) void kb_btri_factor(const LevelArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    btri_factor_body<M, T, ADD>(a, w.y);
}
template <int M, typename T>
__global__ __launch_bounds__(WG) void k_babd_factor(LevelArgs a)
{
    babd_factor_body<M, T>(a, blockIdx.x);
}
template <int M, typename T>
__global__ __launch_bounds__(WG) void kb_babd_factor(const LevelArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    babd_factor_body<M, T>(a, w.y);
}
template <int M, typename T, bool ADD>
__global__ __launch_bounds__(WG) void k_btri_factor_tile(LevelArgs a)
{
    btri_factor_tile_body<M, T, ADD, false>(a, SolveArgs{}, blockIdx.x);
}
template <int M, typename T, bool ADD>
__global__ __launch_bounds__(WG) void kb_btri_factor_tile(const LevelArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    btri_factor_tile_body<M, T, ADD, false>(a, SolveArgs{}, w.y);
}
template <int M, typename T>
__global__ __launch_bounds__(WG) void k_babd_factor_tile(LevelArgs a)
{
    babd_factor_tile_body<M, T, false>(a, SolveArgs{}, blockIdx.x);
}
template <int M, typename T>
__global__ __launch_bounds__(WG) void kb_babd_factor_tile(const LevelArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    babd_factor_tile_body<M, T, false>(a, SolveArgs{}, w.y);
}
// factor-and-solve: factor a level and sweep its right-hand sides forward
template <int M, typename T, bool ADD>
__global__ __launch_bounds__(WG) void k_btri_factor_solve(LevelArgs a, SolveArgs sv)
{
    btri_factor_tile_body<M, T, ADD, true>(a, sv, blockIdx.x);
}
template <int M, typename T>
__global__ __launch_bounds__(WG) void k_babd_factor_solve(LevelArgs a, SolveArgs sv)
{
    babd_factor_tile_body<M, T, true>(a, sv, blockIdx.x);
}
template <int KIND, int M, int KC, typename T, bool ADD>
__global__ __launch_bounds__(WG) void k_fwd(SolveArgs a)
{
    fwd_body<KIND, M, KC, T, ADD>(a, blockIdx.x, blockIdx.y);
}
template <int KIND, int M, int KC, typename T, bool ADD>
__global__ __launch_bounds__(WG) void kb_fwd(const SolveArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const SolveArgs a = tab[w.x];
    fwd_body<KIND, M, KC, T, ADD>(a, w.y, w.z);
}
template <int KIND, int M, int KC, typename T>
__global__ __launch_bounds__(WG) void k_bwd(SolveArgs a)
{
    bwd_body<KIND, M, KC, T>(a, blockIdx.x, blockIdx.y);
}
template <int KIND, int M, int KC, typename T>
__global__ __launch_bounds__(WG) void kb_bwd(const SolveArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const SolveArgs a = tab[w.x];
    bwd_body<KIND, M, KC, T>(a, w.y, w.z);
}

template <typename F>
hipError_t dispatch_M(int M, F &&f)
{
    switch (M) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    default: return hipErrorInvalidValue;
    }
}

template <typename F>
hipError_t dispatch_KC(int KC, F &&f)
{
    return KC == 1 ? f(std::integral_constant<int, 1>{}) : f(std::integral_constant<int, 4>{});
}

inline dim3 grid_for(int M, int64_t p, int nrhs, int KC)
{
    const int64_t gpw = WG / M;
    return dim3((unsigned)((p + gpw - 1) / gpw), (unsigned)((nrhs + KC - 1) / KC), 1);
}

}  // namespace

int groups_per_wg(int M) { return WG / M; }
bool tile_mapping_ok(int M) { return M == 2 || M == 4 || M == 8; }
int partitions_per_wg(int M, bool tile) { return tile ? WG / (M * M) : WG / M; }
int rhs_chunk(int nrhs) { return nrhs == 1 ? 1 : 4; }

template <typename F>
hipError_t dispatch_Mtile(int M, F &&f)
{
    switch (M) {
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_btri_factor(int M, bool f32, bool tile, const LevelArgs &a, hipStream_t s)
{
    const bool add = a.Dadd != nullptr;
    if (tile)
        return dispatch_Mtile(M, [&](auto mc) {
            constexpr int MV = decltype(mc)::value;
            const dim3 grid((unsigned)((a.p + partitions_per_wg(MV, true) - 1) /
                                       partitions_per_wg(MV, true)));
            if (add) {
                if (f32) hipLaunchKernelGGL((k_btri_factor_tile<MV, float, true>), grid, dim3(WG), 0, s, a);
                else hipLaunchKernelGGL((k_btri_factor_tile<MV, double, true>), grid, dim3(WG), 0, s, a);
            } else {
                if (f32) hipLaunchKernelGGL((k_btri_factor_tile<MV, float, false>), grid, dim3(WG), 0, s, a);
                else hipLaunchKernelGGL((k_btri_factor_tile<MV, double, false>), grid, dim3(WG), 0, s, a);
            }
            return hipGetLastError();
        });
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        const dim3 grid = grid_for(MV, a.p, 1, 1);
        if (add) {
            if (f32) hipLaunchKernelGGL((k_btri_factor<MV, float, true>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_btri_factor<MV, double, true>), grid, dim3(WG), 0, s, a);
        } else {
            if (f32) hipLaunchKernelGGL((k_btri_factor<MV, float, false>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_btri_factor<MV, double, false>), grid, dim3(WG), 0, s, a);
        }
        return hipGetLastError();
    });
}

hipError_t launch_babd_factor(int M, bool f32, bool tile, const LevelArgs &a, hipStream_t s)
{
    if (tile)
        return dispatch_Mtile(M, [&](auto mc) {
            constexpr int MV = decltype(mc)::value;
            const dim3 grid((unsigned)((a.p + partitions_per_wg(MV, true) - 1) /
                                       partitions_per_wg(MV, true)));
            if (f32) hipLaunchKernelGGL((k_babd_factor_tile<MV, float>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_babd_factor_tile<MV, double>), grid, dim3(WG), 0, s, a);
            return hipGetLastError();
        });
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        const dim3 grid = grid_for(MV, a.p, 1, 1);
        if (f32) hipLaunchKernelGGL((k_babd_factor<MV, float>), grid, dim3(WG), 0, s, a);
        else hipLaunchKernelGGL((k_babd_factor<MV, double>), grid, dim3(WG), 0, s, a);
        return hipGetLastError();
    });
}

hipError_t launch_factor_solve(int kind, int M, bool f32, const LevelArgs &a, const SolveArgs &sv,
                               hipStream_t s)
{
    if (sv.nrhs < 1 || sv.nrhs > M) return hipErrorInvalidValue;
    return dispatch_Mtile(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        const dim3 grid((unsigned)((a.p + partitions_per_wg(MV, true) - 1) /
                                   partitions_per_wg(MV, true)));
        if (kind == 1) {
            if (f32) hipLaunchKernelGGL((k_babd_factor_solve<MV, float>), grid, dim3(WG), 0, s, a, sv);
            else hipLaunchKernelGGL((k_babd_factor_solve<MV, double>), grid, dim3(WG), 0, s, a, sv);
        } else if (a.Dadd) {
            if (f32) hipLaunchKernelGGL((k_btri_factor_solve<MV, float, true>), grid, dim3(WG), 0, s, a, sv);
            else hipLaunchKernelGGL((k_btri_factor_solve<MV, double, true>), grid, dim3(WG), 0, s, a, sv);
        } else {
            if (f32) hipLaunchKernelGGL((k_btri_factor_solve<MV, float, false>), grid, dim3(WG), 0, s, a, sv);
            else hipLaunchKernelGGL((k_btri_factor_solve<MV, double, false>), grid, dim3(WG), 0, s, a, sv);
        }
        return hipGetLastError();
    });
}

hipError_t launch_factor_batch(int kind, int M, bool f32, bool add, bool tile, const LevelArgs *tab,
                               const int4 *work, int nwg, hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    const dim3 grid(nwg);
    if (tile)
        return dispatch_Mtile(M, [&](auto mc) {
            constexpr int MV = decltype(mc)::value;
            if (kind == 1) {
                if (f32) hipLaunchKernelGGL((kb_babd_factor_tile<MV, float>), grid, dim3(WG), 0, s, tab, work);
                else hipLaunchKernelGGL((kb_babd_factor_tile<MV, double>), grid, dim3(WG), 0, s, tab, work);
            } else if (add) {
                if (f32) hipLaunchKernelGGL((kb_btri_factor_tile<MV, float, true>), grid, dim3(WG), 0, s, tab, work);
                else hipLaunchKernelGGL((kb_btri_factor_tile<MV, double, true>), grid, dim3(WG), 0, s, tab, work);
            } else {
                if (f32) hipLaunchKernelGGL((kb_btri_factor_tile<MV, float, false>), grid, dim3(WG), 0, s, tab, work);
                else hipLaunchKernelGGL((kb_btri_factor_tile<MV, double, false>), grid, dim3(WG), 0, s, tab, work);
            }
            return hipGetLastError();
        });
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        if (kind == 1) {
            if (f32) hipLaunchKernelGGL((kb_babd_factor<MV, float>), grid, dim3(WG), 0, s, tab, work);
            else hipLaunchKernelGGL((kb_babd_factor<MV, double>), grid, dim3(WG), 0, s, tab, work);
        } else if (add) {
            if (f32) hipLaunchKernelGGL((kb_btri_factor<MV, float, true>), grid, dim3(WG), 0, s, tab, work);
            else hipLaunchKernelGGL((kb_btri_factor<MV, double, true>), grid, dim3(WG), 0, s, tab, work);
        } else {
            if (f32) hipLaunchKernelGGL((kb_btri_factor<MV, float, false>), grid, dim3(WG), 0, s, tab, work);
            else hipLaunchKernelGGL((kb_btri_factor<MV, double, false>), grid, dim3(WG), 0, s, tab, work);
        }
        return hipGetLastError();
    });
}

template <int KIND, bool FWD>
static hipError_t launch_solve(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        return dispatch_KC(rhs_chunk(a.nrhs), [&](auto kcc) {
            constexpr int KC = decltype(kcc)::value;
            const dim3 grid = grid_for(MV, a.p, a.nrhs, KC);
            const bool add = KIND == 0 && a.Fadd;
            if (FWD) {
                if (add) {
                    if (f32) hipLaunchKernelGGL((k_fwd<KIND, MV, KC, float, true>), grid, dim3(WG), 0, s, a);
                    else hipLaunchKernelGGL((k_fwd<KIND, MV, KC, double, true>), grid, dim3(WG), 0, s, a);
                } else {
                    if (f32) hipLaunchKernelGGL((k_fwd<KIND, MV, KC, float, false>), grid, dim3(WG), 0, s, a);
                    else hipLaunchKernelGGL((k_fwd<KIND, MV, KC, double, false>), grid, dim3(WG), 0, s, a);
                }
            } else {
                if (f32) hipLaunchKernelGGL((k_bwd<KIND, MV, KC, float>), grid, dim3(WG), 0, s, a);
                else hipLaunchKernelGGL((k_bwd<KIND, MV, KC, double>), grid, dim3(WG), 0, s, a);
            }
            return hipGetLastError();
        });
    });
}

hipError_t launch_btri_fwd(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return launch_solve<0, true>(M, f32, a, s);
}
hipError_t launch_btri_bwd(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return launch_solve<0, false>(M, f32, a, s);
}
hipError_t launch_babd_fwd(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return launch_solve<1, true>(M, f32, a, s);
}
hipError_t launch_babd_bwd(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return launch_solve<1, false>(M, f32, a, s);
}

template <int KIND>
static hipError_t launch_solve_batch_k(bool fwd, int M, bool f32, bool add, int KC,
                                       const SolveArgs *tab, const int4 *work, int nwg,
                                       hipStream_t s)
{
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        return dispatch_KC(KC, [&](auto kcc) {
            constexpr int K = decltype(kcc)::value;
            const dim3 grid(nwg);
            if (fwd) {
                if (KIND == 0 && add) {
                    if (f32) hipLaunchKernelGGL((kb_fwd<KIND, MV, K, float, true>), grid, dim3(WG), 0, s, tab, work);
                    else hipLaunchKernelGGL((kb_fwd<KIND, MV, K, double, true>), grid, dim3(WG), 0, s, tab, work);
                } else {
                    if (f32) hipLaunchKernelGGL((kb_fwd<KIND, MV, K, float, false>), grid, dim3(WG), 0, s, tab, work);
                    else hipLaunchKernelGGL((kb_fwd<KIND, MV, K, double, false>), grid, dim3(WG), 0, s, tab, work);
                }
            } else {
                if (f32) hipLaunchKernelGGL((kb_bwd<KIND, MV, K, float>), grid, dim3(WG), 0, s, tab, work);
                else hipLaunchKernelGGL((kb_bwd<KIND, MV, K, double>), grid, dim3(WG), 0, s, tab, work);
            }
            return hipGetLastError();
        });
    });
}

hipError_t launch_solve_batch(int kind, bool fwd, int M, bool f32, bool add, int KC,
                              const SolveArgs *tab, const int4 *work, int nwg, hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    return kind == 0 ? launch_solve_batch_k<0>(fwd, M, f32, add, KC, tab, work, nwg, s)
                     : launch_solve_batch_k<1>(fwd, M, f32, add, KC, tab, work, nwg, s);
}

}  // namespace pf
