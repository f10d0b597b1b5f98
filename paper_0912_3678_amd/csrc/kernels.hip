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
// of M consecutive lanes (M = block size; 64/M partitions per wave).  In the
// factor kernels lane j holds column j of every block it works on; in the
// solve kernels lane i holds row i.  Left operands of block products go
// through the group's own slice of LDS.  A group never leaves its wave, so
// the only ordering needed between an LDS write and the reads of the other
// lanes is the in-order LDS pipe of the wave plus a compiler fence
// (wave_sync); no workgroup barrier is used.
//
// Memory discipline inside the chain loops: every load and store is issued
// unconditionally (load indices are clamped to a valid block and the values
// masked afterwards; stores of inactive iterations are redirected to a small
// dump buffer) and the zero-pivot report is deferred to the end.  With no
// memory operation under a branch, the compiler's wait counters stay exact:
// a row waits for the loads it needs, never for the stores of earlier rows
// (on this architecture stores and loads share one in-order counter).
//
// Factor storage: per block row g, column-major M x M blocks E (inverse of
// the eliminated pivot block D'), X = E A(g,g+1), Zh (left spike column) and
// R (left spike row) -- exactly the quantities the solve needs.
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

template <typename T> __device__ __forceinline__ T tabs(T v) { return v < T(0) ? -v : v; }

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

// row i of a column-major M x M block of T
template <int M, typename T>
__device__ __forceinline__ void ld_row(T (&v)[M], const T *__restrict__ blk, int i)
{
#pragma unroll
    for (int l = 0; l < M; ++l) v[l] = blk[i + l * M];
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

// ---- Gauss-Jordan inversion of the pivot block with row partial pivoting --
// Lane j holds column j of D' in d; on return e holds column j of D'^{-1}
// (d is consumed).  At step c every lane publishes its current column in the
// group's LDS scratch SG and reads column c; the pivot is the first index of
// the largest magnitude among rows c..M-1 of that column.  Every lane swaps
// the same two rows of its own columns and eliminates column c above and
// below the pivot.  Branch-free (selects only).  Returns true if a pivot was
// exactly zero.
template <int M, typename T>
__device__ __forceinline__ bool gj_invert(T (&d)[M], T (&e)[M], int j, T *SG)
{
    bool sing = false;
#pragma unroll
    for (int r = 0; r < M; ++r) e[r] = (r == j) ? T(1) : T(0);
#pragma unroll
    for (int c = 0; c < M; ++c) {
        lds_put_col<M, T>(SG, j, d);
        wave_sync();
        T col[M];
#pragma unroll
        for (int r = 0; r < M; ++r) col[r] = SG[r + c * M];
        int pr = c;
        T best = tabs(col[c]);
#pragma unroll
        for (int r = c + 1; r < M; ++r) {
            const T v = tabs(col[r]);
            const bool gt = v > best;
            best = gt ? v : best;
            pr = gt ? r : pr;
        }
#pragma unroll
        for (int r = c + 1; r < M; ++r) {
            const bool sw = (r == pr);
            T a0 = d[c], b0 = d[r];
            d[c] = sw ? b0 : a0;
            d[r] = sw ? a0 : b0;
            a0 = e[c]; b0 = e[r];
            e[c] = sw ? b0 : a0;
            e[r] = sw ? a0 : b0;
            a0 = col[c]; b0 = col[r];
            col[c] = sw ? b0 : a0;
            col[r] = sw ? a0 : b0;
        }
        const T pv = col[c];
        sing = sing || (pv == T(0));
        const T inv = T(1) / pv;
        const T dc = d[c] * inv, ec = e[c] * inv;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            if (r == c) continue;
            d[r] = fma(-col[r], dc, d[r]);
            e[r] = fma(-col[r], ec, e[r]);
        }
        d[c] = dc;
        e[c] = ec;
        wave_sync();
    }
    return sing;
}

// ---------------------------------------------------------------------------
// Block tridiagonal factor: one level.  ADD: the diagonal blocks are the sum
// of two arrays (the two neighbours' contributions of the level above).
template <int M, typename T, bool ADD>
__global__ __launch_bounds__(WG) void k_btri_factor(LevelArgs a)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, j = tid % M;
    __shared__ __align__(16) T sA[GPW][M * M];
    __shared__ __align__(16) T sR[GPW][M * M];
    __shared__ __align__(16) T sG[GPW][M * M];
    T *SA = sA[grp], *SR = sR[grp], *SG = sG[grp];

    const int64_t nb = a.nb;
    const int64_t part = (int64_t)blockIdx.x * GPW + grp;
    const Geo G = geometry<0>(nb, a.p, part);
    T *E = (T *)a.E, *R = (T *)a.R, *Zs = (T *)a.Z, *Xs = (T *)a.X;
    T *dump = (T *)a.dump + tid * M;

    T d[M], z[M], rc[M], a1[M];
    zero<M, T>(d); zero<M, T>(z); zero<M, T>(rc); zero<M, T>(a1);
    if (G.valid) {
        ld_vec<M, T>(d, a.D + G.start * MM + j * M);
        if constexpr (ADD) add_vec<M, T>(d, a.Dadd + G.start * MM + j * M);
    }
    if (G.hasL) {
        ld_vec<M, T>(z, a.Lo + (G.start - 1) * MM + j * M);   // A(g_1, sL)
        ld_vec<M, T>(rc, a.Up + (G.start - 1) * MM + j * M);  // A(sL, g_1)
    }
    lds_put_col<M, T>(SR, j, rc);
    wave_sync();
    unsigned long long bad = ~0ull;

    for (int k = 0; k < G.kmax; ++k) {
        const bool act = k < G.len;
        const int64_t g = G.start + k;
        const bool nxt = act && (g + 1 < nb);
        const int64_t gl = nxt ? g : 0, gd = nxt ? g + 1 : 0;
        T up[M], lo[M], dn[M];
        ld_vec<M, T>(up, a.Up + gl * MM + j * M);
        ld_vec<M, T>(lo, a.Lo + gl * MM + j * M);
        ld_vec<M, T>(dn, a.D + gd * MM + j * M);
        if constexpr (ADD) add_vec<M, T>(dn, a.Dadd + gd * MM + j * M);
        mask<M, T>(up, nxt);
        mask<M, T>(lo, nxt);
        mask<M, T>(dn, nxt);

        T e[M], dw[M];
#pragma unroll
        for (int r = 0; r < M; ++r) dw[r] = d[r];
        const bool sing = gj_invert<M, T>(dw, e, j, SG);
        const unsigned long long code = status_code(a.level, g);
        bad = (act && sing && code < bad) ? code : bad;
        st_fac<M, T>(act ? E + g * MM + j * M : dump, e);
        lds_put_col<M, T>(SA, j, e);
        wave_sync();
        T x[M], zh[M];
        lds_gemv2<M, T>(SA, up, z, x, zh);          // X_k, Zh_k
        st_fac<M, T>(act ? Xs + g * MM + j * M : dump, x);
        st_fac<M, T>(act ? Zs + g * MM + j * M : dump, zh);
        T t1[M], rn[M];
        lds_gemv2<M, T>(SR, zh, x, t1, rn);         // R_k Zh_k, R_k X_k
        st_fac<M, T>((act && G.hasL) ? R + g * MM + j * M : dump, rc);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            a1[r] = act ? a1[r] - t1[r] : a1[r];
            rc[r] = act ? -rn[r] : rc[r];
        }
        wave_sync();
        lds_put_col<M, T>(SR, j, rc);
        lds_put_col<M, T>(SA, j, lo);
        wave_sync();
        T dl[M], zl[M];
        lds_gemv2<M, T>(SA, x, zh, dl, zl);         // Lo X_k, Lo Zh_k
#pragma unroll
        for (int r = 0; r < M; ++r) {
            d[r] = act ? dn[r] - dl[r] : d[r];
            z[r] = act ? -zl[r] : z[r];
        }
        wave_sync();
    }
    if (bad != ~0ull) atomicMin(a.status, bad);
    // contributions to the reduced matrix (eq. (redmatr)); separator j sits
    // between partitions j and j+1
    if (G.hasR) {
        double *o = a.nD + part * MM + j * M;
#pragma unroll
        for (int r = 0; r < M; ++r) o[r] = (double)d[r];        // D[sR] + alpha_2
        if (G.hasL) {
            double *ob = a.nLo + (part - 1) * MM + j * M;
#pragma unroll
            for (int r = 0; r < M; ++r) ob[r] = (double)z[r];   // beta
        }
    }
    if (G.hasL) {
        double *oa = a.nDadd + (part - 1) * MM + j * M;
#pragma unroll
        for (int r = 0; r < M; ++r) oa[r] = (double)a1[r];      // alpha_1
        if (G.hasR) {
            double *og = a.nUp + (part - 1) * MM + j * M;
#pragma unroll
            for (int r = 0; r < M; ++r) og[r] = (double)rc[r];  // gamma
        }
    }
}

// ---------------------------------------------------------------------------
// Bidiagonal-plus-corner factor: one level.  Separators s_0 = 0 < s_1 < ... <
// s_p = nb-1; partition `part` lies between s_part and s_{part+1}.  The
// reduced matrix (eq. (redmatr1) with gamma = 0) has the same form:
// diagonal D[s_i], sub-diagonal beta, corner unchanged.
template <int M, typename T>
__global__ __launch_bounds__(WG) void k_babd_factor(LevelArgs a)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, j = tid % M;
    __shared__ __align__(16) T sA[GPW][M * M];
    __shared__ __align__(16) T sG[GPW][M * M];
    T *SA = sA[grp], *SG = sG[grp];

    const int64_t part = (int64_t)blockIdx.x * GPW + grp;
    const Geo G = geometry<1>(a.nb, a.p, part);
    T *E = (T *)a.E, *Zs = (T *)a.Z;
    T *dump = (T *)a.dump + tid * M;

    T z[M];
    zero<M, T>(z);
    if (G.valid) ld_vec<M, T>(z, a.Lo + (G.start - 1) * MM + j * M);   // A(g_1, sL)
    unsigned long long bad = ~0ull;

    for (int k = 0; k < G.kmax; ++k) {
        const bool act = k < G.len;
        const int64_t g = G.start + k;
        const int64_t gc = act ? g : 0;
        T d[M], lo[M];
        ld_vec<M, T>(d, a.D + gc * MM + j * M);
        ld_vec<M, T>(lo, a.Lo + gc * MM + j * M);                      // A(g+1, g)
        T e[M];
        const bool sing = gj_invert<M, T>(d, e, j, SG);
        const unsigned long long code = status_code(a.level, g);
        bad = (act && sing && code < bad) ? code : bad;
        st_fac<M, T>(act ? E + g * MM + j * M : dump, e);
        lds_put_col<M, T>(SA, j, e);
        wave_sync();
        T zh[M];
        lds_gemv<M, T>(SA, z, zh);                  // Zh_k = E_k Z'_k
        st_fac<M, T>(act ? Zs + g * MM + j * M : dump, zh);
        wave_sync();
        lds_put_col<M, T>(SA, j, lo);
        wave_sync();
        T zl[M];
        lds_gemv<M, T>(SA, zh, zl);                 // A(g+1,g) Zh_k
#pragma unroll
        for (int r = 0; r < M; ++r) z[r] = act ? -zl[r] : z[r];
        wave_sync();
    }
    if (bad != ~0ull) atomicMin(a.status, bad);
    if (G.valid) {
        const int64_t sR = G.start + G.len;
        double *ob = a.nLo + part * MM + j * M;
#pragma unroll
        for (int r = 0; r < M; ++r) ob[r] = (double)z[r];                // beta
        const double *ds = a.D + sR * MM + j * M;
        double *od = a.nD + (part + 1) * MM + j * M;
#pragma unroll
        for (int r = 0; r < M; ++r) od[r] = ds[r];
        if (part == 0) {
            double *o0 = a.nD + j * M;
            double *oc = a.nC + j * M;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                o0[r] = a.D[j * M + r];
                oc[r] = a.C[j * M + r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Forward sweep of a solve (the F solve): t_k and the reduced right-hand side.
// Lane i owns row i of KC right-hand-side columns.  ADD: the right-hand side
// is the sum of two arrays (reduced levels of block tridiagonal matrices).
template <int KIND, int M, int KC, typename T, bool ADD>
__global__ __launch_bounds__(WG) void k_fwd(SolveArgs a)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, i = tid % M;
    __shared__ __align__(16) T sV[GPW][KC * M];
    T *SV = sV[grp];
    const int64_t part = (int64_t)blockIdx.x * GPW + grp;
    const Geo G = geometry<KIND>(a.nb, a.p, part);
    const int c0 = blockIdx.y * KC;
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
        if (G.valid && c < kc) {
            double v = a.F[G.start * M + i + col[c] * a.ldf];
            if constexpr (ADD) v += a.Fadd[G.start * M + i + col[c] * a.ldf];
            fp[c] = (T)v;
        }
    }
    for (int k = 0; k < G.kmax; ++k) {
        const bool act = k < G.len;
        const int64_t g = G.start + k;
        const bool nxt = act && (g + 1 < a.nb);
        const int64_t ge = act ? g : 0, gn = nxt ? g : 0;
        T er[M], lr[M], rr[M], fn[KC];
        ld_row<M, T>(er, E + ge * MM, i);
        ld_row_d<M, T>(lr, a.Lo + gn * MM, i);
        if constexpr (KIND == 0) {
            ld_row<M, T>(rr, R + ((act && G.hasL) ? g : 0) * MM, i);
            mask<M, T>(rr, act && G.hasL);
        }
        mask<M, T>(lr, nxt);
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            double v = a.F[(gn + (nxt ? 1 : 0)) * M + i + col[c] * a.ldf];
            if constexpr (ADD) v += a.Fadd[(gn + (nxt ? 1 : 0)) * M + i + col[c] * a.ldf];
            fn[c] = nxt ? (T)v : T(0);
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) SV[i + c * M] = fp[c];
        wave_sync();
        T t[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T s = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) s = fma(er[l], SV[l + c * M], s);
            t[c] = s;
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            double *dst = (act && c < kc) ? a.Y + g * M + i + col[c] * a.ldy : dump;
            *dst = (double)t[c];
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) SV[i + c * M] = t[c];
        wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T sl = T(0), sr = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                const T tv = SV[l + c * M];
                sl = fma(lr[l], tv, sl);
                if constexpr (KIND == 0) sr = fma(rr[l], tv, sr);
            }
            fp[c] = act ? fn[c] - sl : fp[c];
            if constexpr (KIND == 0) gl[c] = act ? gl[c] - sr : gl[c];
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
__global__ __launch_bounds__(WG) void k_bwd(SolveArgs a)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, i = tid % M;
    __shared__ __align__(16) T sV[GPW][KC * M];
    __shared__ __align__(16) T sL[GPW][KC * M];
    T *SV = sV[grp], *SL = sL[grp];
    const int64_t part = (int64_t)blockIdx.x * GPW + grp;
    const Geo G = geometry<KIND>(a.nb, a.p, part);
    const int c0 = blockIdx.y * KC;
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
        SL[i + c * M] = xl;
        SV[i + c * M] = xr;
    }
    wave_sync();
    for (int k = G.kmax - 1; k >= 0; --k) {
        const bool act = k < G.len;
        const int64_t g = G.start + k;
        const int64_t ge = act ? g : 0;
        T zr[M], xrw[M], t[KC];
        ld_row<M, T>(zr, Zs + ge * MM, i);
        if constexpr (KIND == 0) ld_row<M, T>(xrw, Xs + ge * MM, i);
#pragma unroll
        for (int c = 0; c < KC; ++c) t[c] = (T)a.Y[ge * M + i + col[c] * a.ldy];
        T xk[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T s = t[c];
#pragma unroll
            for (int l = 0; l < M; ++l) {
                s = fma(-zr[l], SL[l + c * M], s);
                if constexpr (KIND == 0) s = fma(-xrw[l], SV[l + c * M], s);
            }
            xk[c] = s;
        }
        if constexpr (KIND == 0) wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            double *dst = (act && c < kc) ? a.Y + g * M + i + col[c] * a.ldy : dump;
            *dst = (double)xk[c];
            if constexpr (KIND == 0) SV[i + c * M] = act ? xk[c] : SV[i + c * M];
        }
        if constexpr (KIND == 0) wave_sync();
    }
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

inline dim3 grid_for(int M, int64_t p, int nrhs, int KC)
{
    const int64_t gpw = WG / M;
    return dim3((unsigned)((p + gpw - 1) / gpw), (unsigned)((nrhs + KC - 1) / KC), 1);
}

}  // namespace

hipError_t launch_btri_factor(int M, bool f32, const LevelArgs &a, hipStream_t s)
{
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        const dim3 grid = grid_for(MV, a.p, 1, 1);
        if (a.Dadd) {
            if (f32) hipLaunchKernelGGL((k_btri_factor<MV, float, true>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_btri_factor<MV, double, true>), grid, dim3(WG), 0, s, a);
        } else {
            if (f32) hipLaunchKernelGGL((k_btri_factor<MV, float, false>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_btri_factor<MV, double, false>), grid, dim3(WG), 0, s, a);
        }
        return hipGetLastError();
    });
}

hipError_t launch_babd_factor(int M, bool f32, const LevelArgs &a, hipStream_t s)
{
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        const dim3 grid = grid_for(MV, a.p, 1, 1);
        if (f32) hipLaunchKernelGGL((k_babd_factor<MV, float>), grid, dim3(WG), 0, s, a);
        else hipLaunchKernelGGL((k_babd_factor<MV, double>), grid, dim3(WG), 0, s, a);
        return hipGetLastError();
    });
}

template <int KIND, int M, int KC, typename T>
static void launch_fwd_kernel(const SolveArgs &a, dim3 grid, hipStream_t s)
{
    if (KIND == 0 && a.Fadd)
        hipLaunchKernelGGL((k_fwd<KIND, M, KC, T, true>), grid, dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((k_fwd<KIND, M, KC, T, false>), grid, dim3(WG), 0, s, a);
}

template <int KIND, bool FWD>
static hipError_t launch_solve(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        if (a.nrhs == 1) {
            const dim3 grid = grid_for(MV, a.p, a.nrhs, 1);
            if (FWD) {
                if (f32) launch_fwd_kernel<KIND, MV, 1, float>(a, grid, s);
                else launch_fwd_kernel<KIND, MV, 1, double>(a, grid, s);
            } else {
                if (f32) hipLaunchKernelGGL((k_bwd<KIND, MV, 1, float>), grid, dim3(WG), 0, s, a);
                else hipLaunchKernelGGL((k_bwd<KIND, MV, 1, double>), grid, dim3(WG), 0, s, a);
            }
        } else {
            const dim3 grid = grid_for(MV, a.p, a.nrhs, 4);
            if (FWD) {
                if (f32) launch_fwd_kernel<KIND, MV, 4, float>(a, grid, s);
                else launch_fwd_kernel<KIND, MV, 4, double>(a, grid, s);
            } else {
                if (f32) hipLaunchKernelGGL((k_bwd<KIND, MV, 4, float>), grid, dim3(WG), 0, s, a);
                else hipLaunchKernelGGL((k_bwd<KIND, MV, 4, double>), grid, dim3(WG), 0, s, a);
            }
        }
        return hipGetLastError();
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

}  // namespace pf
