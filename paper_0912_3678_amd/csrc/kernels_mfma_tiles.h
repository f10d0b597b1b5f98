// Partition-method kernels on the matrix cores for 16 x 16 and 32 x 32 blocks
// (gfx950): the block tridiagonal factor kernel for both sizes (every level),
// the factor kernel for 16 x 16 blocks of the bidiagonal-plus-corner form
// (every level, further below) and the forward sweep and back substitution
// for both sizes.  Every body is templated on the arithmetic type V: FP64
// (v_mfma_f64_16x16x4f64; kernels_mfma_tiles.hip instantiates it) or FP32
// with FP32 accumulation (v_mfma_f32_16x16x4f32, the finest level of
// PF_FP32_IR; kernels_mfma_tiles32.hip).  The matrix, the right-hand sides,
// the solutions and the reduced system stay FP64 in memory (converted in
// registers); the factors E, X, Zh, R are stored in V.
//
// Block tridiagonal factor: one partition per wave.  The pivot blocks are
// inverted by the Gauss-Jordan exchange steps of kernels_gj.h with sixteen
// entries per lane for 32 x 32 blocks (lane (r, g) holds row r, columns
// 16g .. 16g+15) and four for 16 x 16 blocks.  The six block products of a chain row
// -- X = E A(g,g+1), Zh = E Z', D'_{k+1} = D[g+1] - A(g+1,g) X,
// Z'_{k+1} = -A(g+1,g) Zh and the spike-row updates -- run on the matrix
// cores as 2 x 2 tiles of 16 x 16, each tile product four
// v_mfma_f64_16x16x4f64 (K = 4 each).
//
// "Quad" layout: of an M x M matrix Y (T = M / 16 tiles of 16 a side), lane l
// (n = l & 15, m = l >> 4) holds Y(16I + rho(m, q), 16J + n) for tiles I, J < T
// and q = 0..3 -- the result layout of the instruction for each tile, which
// differs between the types: rho(m, q) = m + 4q for the FP64 instruction and
// 4m + q for the FP32 one (measured on gfx950).  Instruction h of tile
// product (I, K) x (K, J) takes the K indices 16K + rho(m', h) of lane group m'
// (the order in which a product sums over K is free): the A operand
// A(16I + n, 16K + rho(m, h)), entry (K, I, h) of the quad of A^T, and the B
// operand B(16K + rho(m, h), 16J + n), entry (K, J, h) of the quad of B; so a
// product's result is the next product's right operand as it stands, and the
// left operand of a transposed product, and the spike rows are carried
// transposed (R^T, alpha_1^T).  The
// inverse enters through LDS (its transpose's quad read from the logical rows
// the exchange steps leave); D' goes back to the inversion layout through
// LDS.  The operands of a row are requested at the top of the row: the
// inversion covers their latency.  Outputs and recurrences are those of the
// other factor kernels.  The accumulators live in the matrix cores' own
// registers (this file is compiled without the VGPR form).
#pragma once
#include "kernels_gj.h"

namespace pf {
namespace {

// the four accumulator entries of a lane, per arithmetic type
template <typename V> struct VT;
template <> struct VT<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
};
template <> struct VT<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
};

// C + A B for one 16 x 16 x 4 step (one A and one B entry per lane)
__device__ __forceinline__ VT<double>::v4 mfma4(double a, double b, VT<double>::v4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ VT<float>::v4 mfma4(float a, float b, VT<float>::v4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// row of a tile that entry q of lane group m holds (see the quad layout)
template <typename V> __device__ __forceinline__ constexpr int qrow(int m, int q)
{
    return sizeof(V) == 8 ? m + 4 * q : 4 * m + q;
}

// element loads from raw buffers: S is the type in memory
template <typename S> __device__ __forceinline__ S buf_ld_t(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ double buf_ld_t<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return buf_ld(r, off);
}
template <> __device__ __forceinline__ float buf_ld_t<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

constexpr int kM = 32;   // factor kernel for 32 x 32 blocks
template <typename V> constexpr int kRS = kM + kPad<V>;   // its padded LDS row stride

template <int T, typename V = double> struct QuadT {
    typename VT<V>::v4 t[T][T];   // [I][J], entry q = row rho(m, q) of the tile, column n
};

template <int T, typename V = double> __device__ __forceinline__ QuadT<T, V> qzero()
{
    QuadT<T, V> z;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J) z.t[I][J] = typename VT<V>::v4{V(0), V(0), V(0), V(0)};
    return z;
}
template <int T, typename V> __device__ __forceinline__ QuadT<T, V> qneg(const QuadT<T, V> &a)
{
    QuadT<T, V> z;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J) z.t[I][J] = -a.t[I][J];
    return z;
}

// C + A B; aT = quad of A^T, b = quad of B
template <int T, typename V>
__device__ __forceinline__ QuadT<T, V> mmq(const QuadT<T, V> &aT, const QuadT<T, V> &b, QuadT<T, V> c)
{
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J)
#pragma unroll
            for (int K = 0; K < T; ++K)
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    c.t[I][J] = mfma4(aT.t[K][I][h], b.t[K][J][h], c.t[I][J]);
    return c;
}

// quad of a column-major M x M block of S at byte offset base of resource rs,
// in V (TR: the quad of its transpose; on a row-major block the roles swap)
template <bool TR, int T, typename V, typename S = double>
__device__ __forceinline__ QuadT<T, V> qload(__amdgpu_buffer_rsrc_t rs, uint32_t base, int m, int n)
{
    constexpr int M = 16 * T;
    QuadT<T, V> y;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * I + qrow<V>(m, q), col = 16 * J + n;
                const int e = TR ? col + M * row : row + M * col;
                y.t[I][J][q] = (V)buf_ld_t<S>(rs, base + (uint32_t)(e * (int)sizeof(S)));
            }
    return y;
}
// quad into a row-major factor block of V (TR: store the transpose's entries)
template <bool TR, int T, typename V>
__device__ __forceinline__ void qstore_t(__amdgpu_buffer_rsrc_t rs, uint32_t base, bool keep,
                                         const QuadT<T, V> &y, int m, int n)
{
    constexpr int M = 16 * T;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * I + qrow<V>(m, q), col = 16 * J + n;
                const int e = TR ? col * M + row : row * M + col;
                buf_st(rs, keep ? base + (uint32_t)(e * (int)sizeof(V)) : kOffNone, y.t[I][J][q]);
            }
}
// quad (any T) into a column-major FP64 block of global memory
template <bool TR, int T, typename V>
__device__ __forceinline__ void qstore_gt(double *p, const QuadT<T, V> &y, int m, int n)
{
    constexpr int M = 16 * T;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * I + qrow<V>(m, q), col = 16 * J + n;
                p[TR ? col + M * row : row + M * col] = (double)y.t[I][J][q];
            }
}

// A column tile: an M x 16 block of right-hand sides of one block row in the
// quad layout (lane (m, n): rows 16I + rho(m, q) of column n).
template <int T, typename V = double> struct ColT {
    typename VT<V>::v4 t[T];   // [I], entry q = row 16I + rho(m, q), column n of the tile
};

template <int T, typename V = double> __device__ __forceinline__ ColT<T, V> czero()
{
    ColT<T, V> c;
#pragma unroll
    for (int I = 0; I < T; ++I) c.t[I] = typename VT<V>::v4{V(0), V(0), V(0), V(0)};
    return c;
}
// C + A B for one tile; aT = quad of A^T
template <int T, typename V>
__device__ __forceinline__ ColT<T, V> mmc(const QuadT<T, V> &aT, const ColT<T, V> &b, ColT<T, V> c)
{
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int K = 0; K < T; ++K)
#pragma unroll
            for (int h = 0; h < 4; ++h) c.t[I] = mfma4(aT.t[K][I][h], b.t[K][h], c.t[I]);
    return c;
}
// tile of a column-major FP64 array, in V (p: row 0 of the block row, column
// n of the tile; zero when the column does not exist)
template <int T, typename V = double>
__device__ __forceinline__ ColT<T, V> cload(const double *p, bool act, int m)
{
    ColT<T, V> c;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int q = 0; q < 4; ++q) c.t[I][q] = act ? (V)p[16 * I + qrow<V>(m, q)] : V(0);
    return c;
}
template <int T, typename V>
__device__ __forceinline__ void cstore(double *p, bool act, const ColT<T, V> &c, int m)
{
    if (!act) return;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int q = 0; q < 4; ++q) p[16 * I + qrow<V>(m, q)] = (double)c.t[I][q];
}
template <int T, typename V>
__device__ __forceinline__ ColT<T, V> cadd(ColT<T, V> a, const ColT<T, V> &b)
{
#pragma unroll
    for (int I = 0; I < T; ++I) a.t[I] += b.t[I];
    return a;
}

// RHS (one tile, M = 16): up to 16 right-hand sides swept forward in the same
// pass -- t_k = E_k f'_k, f'_{k+1} = f[g+1] - A(g+1,g) t_k, g_sL -= R_k t_k.
template <int T, bool ADD, bool RHS = false, typename V = double>
__device__ __forceinline__ void btri_mfmat_body(const LevelArgs &a, const SolveArgs &sv,
                                                int64_t part, int lane, V *lds)
{
    static_assert(!RHS || T == 1, "the fused forward sweep is built for 16 x 16 blocks");
    using Q = QuadT<T, V>;
    using C1 = ColT<1, V>;
    constexpr int M = 16 * T, E = T == 1 ? 4 : 16, RS = M + kPad<V>;
    constexpr size_t MM = (size_t)M * M;
    constexpr uint32_t BB = MM * 8;                   // an FP64 block of the matrix
    constexpr uint32_t BF = MM * sizeof(V);           // a factor block
    // inversion role: row r, columns 16g ..; matrix-core role: (m, n)
    const int r = lane % M, gc = lane / M, c0 = gc * E;
    const int m = lane >> 4, n = lane & 15;
    V *S0 = lds;              // tableau
    V *SE = S0 + M * RS;      // E by logical rows; then D' handed over

    const int64_t nb = a.nb;
    const Geo G = geometry_wave<0>(nb, a.p, part, a.sep);
    const int64_t gb = G.start > 0 ? G.start - 1 : 0;
    const uint64_t nr = (uint64_t)(nb - gb), nr1 = nb - 1 > gb ? (uint64_t)(nb - 1 - gb) : 0;
    const auto rD = buf_rsrc(a.D + gb * MM, nr * BB);
    const auto rDa = buf_rsrc(ADD ? a.Dadd + gb * MM : a.D, ADD ? nr * BB : 0);
    const auto rL = buf_rsrc(a.Lo + gb * MM, nr1 * BB);
    const auto rU = buf_rsrc(a.Up + gb * MM, nr1 * BB);
    const auto rE = buf_rsrc((V *)a.E + gb * MM, nr * BF);
    const auto rR = buf_rsrc((V *)a.R + gb * MM, nr * BF);
    const auto rZ = buf_rsrc((V *)a.Z + gb * MM, nr * BF);
    const auto rX = buf_rsrc((V *)a.X + gb * MM, nr * BF);
    const uint32_t rel = (uint32_t)(G.start - gb);

    // D'_1 in the inversion layout
    V d[E];
    {
        const uint32_t o = rel * BB + (uint32_t)(r + M * c0) * 8;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            double v = buf_ld(rD, o + (uint32_t)(e * M * 8));
            if constexpr (ADD) v += buf_ld(rDa, o + (uint32_t)(e * M * 8));
            d[e] = (V)v;
        }
    }
    // right-hand-side column n of the tiles; f'_1 = f[g_1], g_sL
    const bool act = RHS && n < sv.nrhs;
    const bool fadd = RHS && sv.Fadd != nullptr;
    const int64_t cf = (int64_t)(act ? n : 0) * sv.ldf, cy = (int64_t)(act ? n : 0) * sv.ldy;
    const int64_t cn = (int64_t)(act ? n : 0) * sv.ldn;
    auto load_f = [&](int64_t g, bool ok) {
        C1 c = cload<1, V>(sv.F + g * M + cf, act && ok, m);
        return fadd ? cadd<1>(c, cload<1, V>(sv.Fadd + g * M + cf, act && ok, m)) : c;
    };
    C1 fp = czero<1, V>(), gl = czero<1, V>();
    if constexpr (RHS) fp = load_f(G.start, G.valid);
    // Z'_1 = A(g_1, sL), R_1^T = A(sL, g_1)^T, alpha_1^T
    Q z = qzero<T, V>(), rT = qzero<T, V>(), a1 = qzero<T, V>(), dq = qzero<T, V>();
    if (G.hasL) {
        z = qload<false, T, V>(rL, (rel - 1) * BB, m, n);
        rT = qload<true, T, V>(rU, (rel - 1) * BB, m, n);
    }
    if (G.len == 0) {   // an empty partition (enlarged reduced systems): D' of sR is D[sR]
        dq = qload<false, T, V>(rD, rel * BB, m, n);
        if constexpr (ADD) {
            const Q da = qload<false, T, V>(rDa, rel * BB, m, n);
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int J = 0; J < T; ++J) dq.t[I][J] += da.t[I][J];
        }
    }
    unsigned long long bad = ~0ull;

    for (int k = 0; k < G.len; ++k) {
        const uint32_t row = rel + (uint32_t)k;
        // this row's operands, requested before the inversion
        const Q up = qload<false, T, V>(rU, row * BB, m, n);     // A(g,g+1)
        const Q loT = qload<true, T, V>(rL, row * BB, m, n);     // A(g+1,g)^T
        Q dn = qload<false, T, V>(rD, (row + 1) * BB, m, n);     // D[g+1]
        if constexpr (ADD) {
            const Q da = qload<false, T, V>(rDa, (row + 1) * BB, m, n);
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int J = 0; J < T; ++J) dn.t[I][J] += da.t[I][J];
        }
        C1 fn = czero<1, V>();
        if constexpr (RHS) fn = load_f(G.start + k + 1, G.start + k + 1 < nb);   // f[g+1]

        // E_k = D'_k^{-1}
        int sigma = 0, pc[E];
#pragma unroll
        for (int e = 0; e < E; ++e) pc[e] = 0;
        bool sing = false;
        seg_invert<M, E, V>(d, r, gc, S0, sigma, pc, sing, (V)a.tau);
        const unsigned long long code = status_code(a.level, G.start + k);
        bad = (sing && code < bad) ? code : bad;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            SE[sigma * RS + pc[e]] = d[e];
            buf_st(rE, row * BF + (uint32_t)(sigma * M + pc[e]) * (uint32_t)sizeof(V), d[e]);
        }
        wave_sync();
        Q eT;   // quad of E^T: E(16I' + n, 16K' + rho(m, q)) at tile [K'][I']
#pragma unroll
        for (int K = 0; K < T; ++K)
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    eT.t[K][I][q] = SE[(16 * I + n) * RS + 16 * K + qrow<V>(m, q)];

        const Q x = mmq<T>(eT, up, qzero<T, V>());    // X_k = E_k A(g,g+1)
        const Q zh = mmq<T>(eT, z, qzero<T, V>());    // Zh_k = E_k Z'_k
        qstore_t<false, T>(rX, row * BF, true, x, m, n);
        qstore_t<false, T>(rZ, row * BF, true, zh, m, n);
        qstore_t<true, T>(rR, row * BF, G.hasL, rT, m, n);   // R_k (row-major) from R_k^T
        const Q nlo = qneg<T>(loT);
        dq = mmq<T>(nlo, x, dn);                   // D'_{k+1} = D[g+1] - A(g+1,g) X_k
        z = mmq<T>(nlo, zh, qzero<T, V>());        // Z'_{k+1} = -A(g+1,g) Zh_k
        if constexpr (RHS) {
            const C1 tk = mmc<1>(eT, fp, czero<1, V>());              // t_k = E_k f'_k
            cstore<1>(sv.Y + (G.start + k) * M + cy, act, tk, m);
            gl = mmc<1>(qneg<1>(rT), tk, gl);                         // g_sL -= R_k t_k
            fp = mmc<1>(nlo, tk, fn);                                 // f'_{k+1} = f[g+1] - A(g+1,g) t_k
        }
        a1 = mmq<T>(qneg<T>(zh), rT, a1);             // alpha_1^T -= Zh_k^T R_k^T
        rT = mmq<T>(qneg<T>(x), rT, qzero<T, V>());   // R_{k+1}^T = -X_k^T R_k^T

        // D'_{k+1} to the inversion layout
        wave_sync();
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = 0; J < T; ++J)
#pragma unroll
                for (int q = 0; q < 4; ++q) SE[(16 * I + qrow<V>(m, q)) * RS + 16 * J + n] = dq.t[I][J][q];
        wave_sync();
        lds_row<E, V>(d, SE + r * RS + c0);
        wave_sync();
    }
    report_bad(a, bad);
    if (G.hasR) {
        qstore_gt<false, T>(a.nD + part * MM, dq, m, n);                      // D[sR] + alpha_2
        if (G.hasL) qstore_gt<false, T>(a.nLo + (part - 1) * MM, z, m, n);    // beta
    }
    if (G.hasL) {
        qstore_gt<true, T>(a.nDadd + (part - 1) * MM, a1, m, n);              // alpha_1
        if (G.hasR) qstore_gt<true, T>(a.nUp + (part - 1) * MM, rT, m, n);    // gamma
    }
    if constexpr (RHS) {
        if (G.hasR) cstore<1>(sv.nF + part * M + cn, act, fp, m);            // f[sR] - A(sR,g_n) t_n
        if (G.hasL) cstore<1>(sv.nFadd + (part - 1) * M + cn, act, gl, m);   // -sum R_k t_k
    }
}

template <bool ADD, typename V>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(sizeof(V) == 4 ? 2 : 1))) void k_btri_mfma32(LevelArgs a)
{
    __shared__ __align__(16) V lds[2 * kM * kRS<V>];
    btri_mfmat_body<2, ADD, false, V>(a, SolveArgs{}, blockIdx.x, threadIdx.x, lds);
}
template <bool ADD, bool RHS, typename V>
__global__ __launch_bounds__(WG) void k_btri_mfma16(LevelArgs a, SolveArgs sv)
{
    __shared__ __align__(16) V lds[2 * 16 * (16 + kPad<V>)];
    btri_mfmat_body<1, ADD, RHS, V>(a, sv, blockIdx.x, threadIdx.x, lds);
}
// batched: workgroup w serves table entry work[w].x, partition work[w].y
template <bool ADD, typename V>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(sizeof(V) == 4 ? 2 : 1))) void kb_btri_mfma32(const LevelArgs *tab, const int4 *work)
{
    __shared__ __align__(16) V lds[2 * kM * kRS<V>];
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    btri_mfmat_body<2, ADD, false, V>(a, SolveArgs{}, w.y, threadIdx.x, lds);
}
template <bool ADD, typename V>
__global__ __launch_bounds__(WG) void kb_btri_mfma16(const LevelArgs *tab, const int4 *work)
{
    __shared__ __align__(16) V lds[2 * 16 * (16 + kPad<V>)];
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    btri_mfmat_body<1, ADD, false, V>(a, SolveArgs{}, w.y, threadIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Forward sweep and back substitution for M = 16 and 32 with factors of type
// V (any factor kernel's row-major E, X, Zh, R), the right-hand sides in
// column tiles of 16: a tile's M x 16 block of one block row sits in the quad
// layout (lane (m, n): rows 16I + rho(m, q) of column n).  Every block product
// is a chain of 16 x 16 x 4 matrix-core steps whose left operand is a factor
// block's transpose quad, loaded straight from memory, so the factors of a
// block row are read once per CT tiles (the row kernels read them once per
// four columns).  KIND: 0 block tridiagonal, 1 bidiagonal plus corner.
template <int M, int KIND, int CT, bool ADD, typename V = double>
__device__ __forceinline__ void fwdt_body(const SolveArgs &a, int64_t part, int cg, int lane)
{
    constexpr int T = M / 16;
    using Col = ColT<T, V>;
    using Q = QuadT<T, V>;
    constexpr size_t MM = (size_t)M * M;
    constexpr uint32_t BB = MM * 8, BF = MM * sizeof(V);
    const int m = lane >> 4, n = lane & 15;
    const int64_t nb = a.nb;
    const Geo G = geometry_wave<KIND>(nb, a.p, part, a.sep);
    const int64_t gb = G.start > 0 ? G.start - 1 : 0;
    const uint64_t nr = (uint64_t)(nb - gb), nr1 = nb - 1 > gb ? (uint64_t)(nb - 1 - gb) : 0;
    const auto rE = buf_rsrc((const V *)a.E + gb * MM, nr * BF);
    const auto rR = buf_rsrc(KIND == 0 ? (const V *)a.R + gb * MM : (const V *)a.E, KIND == 0 ? nr * BF : 0);
    const auto rL = buf_rsrc(a.Lo + gb * MM, nr1 * BB);
    const uint32_t rel = (uint32_t)(G.start - gb);
    bool act[CT];
    int64_t cf[CT], cy[CT], cn[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        const int c = (cg * CT + j) * 16 + n;
        act[j] = c < a.nrhs;
        cf[j] = (int64_t)(act[j] ? c : 0) * a.ldf;
        cy[j] = (int64_t)(act[j] ? c : 0) * a.ldy;
        cn[j] = (int64_t)(act[j] ? c : 0) * a.ldn;
    }
    Col fp[CT], gl[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        fp[j] = cload<T, V>(a.F + G.start * M + cf[j], act[j] && G.valid, m);
        if constexpr (ADD) fp[j] = cadd<T>(fp[j], cload<T, V>(a.Fadd + G.start * M + cf[j], act[j] && G.valid, m));
        gl[j] = czero<T, V>();
    }
    // 32 x 32 factors with 64 columns: one factor block in registers at a
    // time (t_k for every tile, then R_k, then A(g+1,g)), so that the four
    // tiles' f', t and g fit beside it
    constexpr bool kStaged = M == 32 && CT == 4 && KIND == 0;
    for (int k = 0; kStaged && k < G.len; ++k) {
        const int64_t g = G.start + k;
        const uint32_t row = rel + (uint32_t)k;
        const bool nx = g + 1 < nb;
        Col t[CT];
        {
            const Q eT = qload<false, T, V, V>(rE, row * BF, m, n);
#pragma unroll
            for (int j = 0; j < CT; ++j) t[j] = mmc(eT, fp[j], czero<T, V>());   // t_k = E_k f'_k
        }
#pragma unroll
        for (int j = 0; j < CT; ++j) cstore<T>(a.Y + g * M + cy[j], act[j], t[j], m);
        if (G.hasL) {
            const Q nrt = qneg<T>(qload<false, T, V, V>(rR, row * BF, m, n));
#pragma unroll
            for (int j = 0; j < CT; ++j) gl[j] = mmc(nrt, t[j], gl[j]);         // g_sL -= R_k t_k
        }
        const Q nlo = qneg<T>(qload<true, T, V>(rL, row * BB, m, n));
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            Col fn = cload<T, V>(a.F + (g + 1) * M + cf[j], act[j] && nx, m);
            if constexpr (ADD) fn = cadd<T>(fn, cload<T, V>(a.Fadd + (g + 1) * M + cf[j], act[j] && nx, m));
            fp[j] = mmc(nlo, t[j], fn);                                          // f'_{k+1}
        }
    }
    for (int k = 0; !kStaged && k < G.len; ++k) {
        const int64_t g = G.start + k;
        const uint32_t row = rel + (uint32_t)k;
        const Q eT = qload<false, T, V, V>(rE, row * BF, m, n);     // E_g^T (E row-major)
        const Q nlo = qneg<T>(qload<true, T, V>(rL, row * BB, m, n));   // -A(g+1,g)^T
        const Q nrt = (KIND == 0 && G.hasL) ? qneg<T>(qload<false, T, V, V>(rR, row * BF, m, n)) : qzero<T, V>();
        const bool nx = g + 1 < nb;
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            Col fn = cload<T, V>(a.F + (g + 1) * M + cf[j], act[j] && nx, m);
            if constexpr (ADD) fn = cadd<T>(fn, cload<T, V>(a.Fadd + (g + 1) * M + cf[j], act[j] && nx, m));
            const Col t = mmc(eT, fp[j], czero<T, V>());               // t_k = E_k f'_k
            cstore<T>(a.Y + g * M + cy[j], act[j], t, m);
            fp[j] = mmc(nlo, t, fn);                                 // f'_{k+1} = f[g+1] - A(g+1,g) t_k
            if constexpr (KIND == 0) gl[j] = mmc(nrt, t, gl[j]);     // g_sL -= R_k t_k
        }
    }
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        if (KIND == 0) {
            if (G.hasR) cstore<T>(a.nF + part * M + cn[j], act[j], fp[j], m);
            if (G.hasL) cstore<T>(a.nFadd + (part - 1) * M + cn[j], act[j], gl[j], m);
        } else if (G.valid) {
            cstore<T>(a.nF + (part + 1) * M + cn[j], act[j], fp[j], m);
            if (part == 0) cstore<T>(a.nF + cn[j], act[j], cload<T, V>(a.F + cf[j], act[j], m), m);
        }
    }
}

template <int M, int KIND, int CT, typename V = double>
__device__ __forceinline__ void bwdt_body(const SolveArgs &a, int64_t part, int cg, int lane)
{
    constexpr int T = M / 16;
    using Col = ColT<T, V>;
    using Q = QuadT<T, V>;
    constexpr size_t MM = (size_t)M * M;
    constexpr uint32_t BF = MM * sizeof(V);
    const int m = lane >> 4, n = lane & 15;
    const int64_t nb = a.nb;
    const Geo G = geometry_wave<KIND>(nb, a.p, part, a.sep);
    const int64_t gb = G.start > 0 ? G.start - 1 : 0;
    const uint64_t nr = (uint64_t)(nb - gb);
    const auto rZ = buf_rsrc((const V *)a.Z + gb * MM, nr * BF);
    const auto rX = buf_rsrc(KIND == 0 ? (const V *)a.X + gb * MM : (const V *)a.Z, KIND == 0 ? nr * BF : 0);
    const uint32_t rel = (uint32_t)(G.start - gb);
    const int64_t sR = G.start + G.len;
    const int64_t jl = (KIND == 0) ? part - 1 : part;
    const int64_t jr = (KIND == 0) ? part : part + 1;
    bool act[CT];
    int64_t cy[CT], cn[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        const int c = (cg * CT + j) * 16 + n;
        act[j] = c < a.nrhs;
        cy[j] = (int64_t)(act[j] ? c : 0) * a.ldy;
        cn[j] = (int64_t)(act[j] ? c : 0) * a.ldn;
    }
    Col xl[CT], xn[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        xl[j] = cload<T, V>(a.Xsep + jl * M + cn[j], act[j] && G.hasL, m);
        xn[j] = cload<T, V>(a.Xsep + jr * M + cn[j], act[j] && G.hasR, m);
        // the separators' solution passes through unrounded
        if (G.hasR)
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t o = sR * M + cy[j] + 16 * I + qrow<V>(m, q);
                    if (act[j]) a.Y[o] = a.Xsep[jr * M + cn[j] + 16 * I + qrow<V>(m, q)];
                }
        if (KIND == 1 && G.valid && part == 0 && act[j])
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    a.Y[cy[j] + 16 * I + qrow<V>(m, q)] = a.Xsep[cn[j] + 16 * I + qrow<V>(m, q)];
    }
    if constexpr (KIND == 1) {
        // x_k = t_k - Zh_k x_sL: the rows are independent, 4 / T at a time
        // (all loads first)
        constexpr int R = 4 / T;
        for (int k0 = 0; k0 < G.len; k0 += R) {
            Q nzt[R];
            Col c[R][CT];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const bool ok = k0 + i < G.len;
                nzt[i] = qload<false, T, V, V>(rZ, (rel + (uint32_t)(k0 + i)) * BF, m, n);
#pragma unroll
                for (int j = 0; j < CT; ++j)
                    c[i][j] = cload<T, V>(a.Y + (G.start + k0 + i) * M + cy[j], act[j] && ok, m);
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const bool ok = k0 + i < G.len;
#pragma unroll
                for (int j = 0; j < CT; ++j) {
                    c[i][j] = mmc(qneg<T>(nzt[i]), xl[j], c[i][j]);   // t_k - Zh_k x_sL
                    cstore<T>(a.Y + (G.start + k0 + i) * M + cy[j], act[j] && ok, c[i][j], m);
                }
            }
        }
        return;
    }
    for (int k = G.len - 1; k >= 0; --k) {
        const int64_t g = G.start + k;
        const uint32_t row = rel + (uint32_t)k;
        const Q nzt = qneg<T>(qload<false, T, V, V>(rZ, row * BF, m, n));                            // -Zh_g
        const Q nxt = KIND == 0 ? qneg<T>(qload<false, T, V, V>(rX, row * BF, m, n)) : qzero<T, V>();   // -X_g
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            Col c = cload<T, V>(a.Y + g * M + cy[j], act[j], m);     // t_k
            c = mmc(nzt, xl[j], c);                             // - Zh_k x_sL
            if constexpr (KIND == 0) c = mmc(nxt, xn[j], c);    // - X_k x_{k+1}
            cstore<T>(a.Y + g * M + cy[j], act[j], c, m);
            xn[j] = c;
        }
    }
}

template <int M, int KIND, int CT, bool ADD, typename V>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void k_fwdt(SolveArgs a)
{
    fwdt_body<M, KIND, CT, ADD, V>(a, blockIdx.x, blockIdx.y, threadIdx.x);
}
template <int M, int KIND, int CT, typename V>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void k_bwdt(SolveArgs a)
{
    bwdt_body<M, KIND, CT, V>(a, blockIdx.x, blockIdx.y, threadIdx.x);
}
template <int M, int KIND, int CT, bool ADD, typename V>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void kb_fwdt(const SolveArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const SolveArgs a = tab[w.x];
    fwdt_body<M, KIND, CT, ADD, V>(a, w.y, w.z, threadIdx.x);
}
template <int M, int KIND, int CT, typename V>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void kb_bwdt(const SolveArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const SolveArgs a = tab[w.x];
    bwdt_body<M, KIND, CT, V>(a, w.y, w.z, threadIdx.x);
}

// ---------------------------------------------------------------------------
// Factor kernel for 16 x 16 blocks of the bidiagonal-plus-corner form (FP64,
// every level; RHS: up to 16 right-hand sides swept forward in the same
// pass).  In this form the pivot blocks do not depend on the chain (D' = D),
// so a wave inverts four consecutive blocks of its partition at once --
// sixteen lanes per block, one tableau row per lane, the exchange steps of
// kernels_gj.h -- and then runs the chain of those rows on the matrix cores
// (one 16 x 16 tile per product): Zh_k = E_k Z'_k, t_k = E_k f'_k,
// Z'_{k+1} = -A(g+1,g) Zh_k, f'_{k+1} = f[g+1] - A(g+1,g) t_k.  The first
// row's chain operands are requested before the inversion, which covers
// their latency, and each later row's one row ahead.  Outputs are those of
// the segment kernel (E and Zh row-major; beta, the next diagonal block and
// the reduced right-hand side).
constexpr int kBQ = 4;                              // blocks inverted together
template <typename V> constexpr int kBRS = 16 + kPad<V>;   // padded LDS row stride
template <typename V> constexpr int kBSL = 16 * kBRS<V>;   // one block in LDS
constexpr uint32_t kOffRowNone = 0xFFFFFF80u;       // 128 bytes past every resource

template <bool RHS, typename V = double>
__device__ __forceinline__ void babd_mfma16_body(const LevelArgs &a, const SolveArgs &sv,
                                                 int64_t part, int lane, V *lds)
{
    constexpr int M = 16, E = 16;
    constexpr int BRS = kBRS<V>, BSL = kBSL<V>;
    constexpr size_t MM = (size_t)M * M;
    constexpr uint32_t BB = MM * 8, BF = MM * sizeof(V);
    using Q = QuadT<1, V>;
    using C1 = ColT<1, V>;
    // inversion role: block q of the group, tableau row r; matrix-core role: (m, n)
    const int q = lane / M, r = lane % M;
    const int m = lane >> 4, n = lane & 15;
    V *S0 = lds + q * BSL;             // tableau of block q
    V *SE = lds + (kBQ + q) * BSL;     // E_q by logical rows

    const int64_t nb = a.nb;
    const Geo G = geometry_wave<1>(nb, a.p, part, a.sep);
    const int64_t gb = G.start - 1;         // the left separator (G.start >= 1)
    const uint64_t nr = (uint64_t)(nb - gb), nr1 = nb - 1 > gb ? (uint64_t)(nb - 1 - gb) : 0;
    const auto rD = buf_rsrc(a.D + gb * MM, nr * BB);
    const auto rL = buf_rsrc(a.Lo + gb * MM, nr1 * BB);
    const auto rE = buf_rsrc((V *)a.E + gb * MM, nr * BF);
    const auto rZ = buf_rsrc((V *)a.Z + gb * MM, nr * BF);
    const uint32_t rel = (uint32_t)(G.start - gb);

    const bool act = RHS && n < sv.nrhs;    // right-hand-side column n of the tiles
    const int64_t cf = (int64_t)(act ? n : 0) * sv.ldf, cy = (int64_t)(act ? n : 0) * sv.ldy;
    const int64_t cn = (int64_t)(act ? n : 0) * sv.ldn;

    // Z'_1 = A(g_1, sL), f'_1 = f[g_1]
    Q z = qload<false, 1, V>(rL, (rel - 1) * BB, m, n);
    C1 fp = czero<1, V>();
    if constexpr (RHS) fp = cload<1, V>(sv.F + G.start * M + cf, act && G.valid, m);
    unsigned long long bad = ~0ull;

    for (int k0 = 0; k0 < G.len; k0 += kBQ) {
        const int nq = G.len - k0 < kBQ ? G.len - k0 : kBQ;
        // block q of the group: D[g], row r (column-major block)
        const bool vq = q < nq;
        V d[E];
        {
            const uint32_t o = (rel + (uint32_t)(k0 + q)) * BB + (uint32_t)r * 8;
#pragma unroll
            for (int e = 0; e < E; ++e) d[e] = (V)buf_ld(rD, o + (uint32_t)(e * M * 8));
        }

        // chain operands of the group's first row, A(g+1,g)^T and f[g+1], then
        // one row ahead
        auto load_lo = [&](int k) { return qload<true, 1, V>(rL, (rel + (uint32_t)k) * BB, m, n); };
        auto load_fn = [&](int k) {
            const int64_t g1 = G.start + k + 1;
            return RHS ? cload<1, V>(sv.F + g1 * M + cf, act && k < G.len && g1 < nb, m) : czero<1, V>();
        };
        Q loN = load_lo(k0);
        C1 fnN = load_fn(k0);

        // E = D^{-1} of the group's blocks
        int sigma = 0, pc[E];
#pragma unroll
        for (int e = 0; e < E; ++e) pc[e] = 0;
        bool sing = false;
        seg_invert<M, E, V>(d, r, 0, S0, sigma, pc, sing, (V)a.tau);
        const unsigned long long code = status_code(a.level, G.start + k0 + q);
        bad = (sing && vq && code < bad) ? code : bad;
#pragma unroll
        for (int e = 0; e < E; ++e) SE[sigma * BRS + pc[e]] = d[e];
        wave_sync();
        {
            V er[E];
            lds_row<E, V>(er, SE + r * BRS);
            buf_st_row<E, V>(rE, vq ? (rel + (uint32_t)(k0 + q)) * BF + (uint32_t)(r * M) * (uint32_t)sizeof(V)
                                    : kOffRowNone, er);
        }

        // the chain over the group's rows (matrix-core role)
#pragma unroll
        for (int i = 0; i < kBQ; ++i) {
            if (i < nq) {
                const int64_t g = G.start + k0 + i;
                const uint32_t row = rel + (uint32_t)(k0 + i);
                const V *Ei = lds + (kBQ + i) * BSL;
                Q eT;   // quad of E^T: E(n, rho(m, h))
#pragma unroll
                for (int h = 0; h < 4; ++h) eT.t[0][0][h] = Ei[n * BRS + qrow<V>(m, h)];
                const Q nlo = qneg<1>(loN);   // -A(g+1,g)^T
                const C1 fn = fnN;
                loN = load_lo(k0 + i + 1);
                fnN = load_fn(k0 + i + 1);
                const Q zh = mmq<1>(eT, z, qzero<1, V>());   // Zh_k = E_k Z'_k
                qstore_t<false, 1>(rZ, row * BF, true, zh, m, n);
                z = mmq<1>(nlo, zh, qzero<1, V>());          // Z'_{k+1} = -A(g+1,g) Zh_k
                if constexpr (RHS) {
                    const C1 tk = mmc<1>(eT, fp, czero<1, V>());   // t_k = E_k f'_k
                    cstore<1>(sv.Y + g * M + cy, act, tk, m);
                    fp = mmc<1>(nlo, tk, fn);                      // f'_{k+1} = f[g+1] - A(g+1,g) t_k
                }
            }
        }
        wave_sync();
    }
    report_bad(a, bad);
    if (G.valid) {
        const int64_t sR = G.start + G.len;
        qstore_gt<false, 1>(a.nLo + part * MM, z, m, n);   // beta
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = lane + 64 * i;
            a.nD[(part + 1) * MM + e] = a.D[sR * MM + e];
            if (part == 0) {
                a.nD[e] = a.D[e];
                a.nC[e] = a.C[e];
            }
        }
        if constexpr (RHS) {
            cstore<1>(sv.nF + (part + 1) * M + cn, act, fp, m);
            if (part == 0 && act)
#pragma unroll
                for (int h = 0; h < 4; ++h) sv.nF[cn + qrow<V>(m, h)] = sv.F[cf + qrow<V>(m, h)];
        }
    }
}

template <bool RHS, typename V>
__global__ __launch_bounds__(WG) void k_babd_mfma16(LevelArgs a, SolveArgs sv)
{
    __shared__ __align__(16) V lds[2 * kBQ * kBSL<V>];
    babd_mfma16_body<RHS, V>(a, sv, blockIdx.x, threadIdx.x, lds);
}
// batched (factor only): workgroup w serves table entry work[w].x, partition work[w].y
template <typename V>
__global__ __launch_bounds__(WG) void kb_babd_mfma16(const LevelArgs *tab, const int4 *work)
{
    __shared__ __align__(16) V lds[2 * kBQ * kBSL<V>];
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    babd_mfma16_body<false, V>(a, SolveArgs{}, w.y, threadIdx.x, lds);
}

template <typename F>
hipError_t dispatch_CT(int cols, F &&f)
{
    return cols <= 16   ? f(std::integral_constant<int, 1>{})
           : cols <= 32 ? f(std::integral_constant<int, 2>{})
                        : f(std::integral_constant<int, 4>{});
}
template <typename F>
hipError_t dispatch_T(int M, F &&f)
{
    if (M == 16) return f(std::integral_constant<int, 16>{});
    if (M == 32) return f(std::integral_constant<int, 32>{});
    return hipErrorInvalidValue;
}

// The launches of this file's kernels for arithmetic type V (the public
// launchers of pf_internal.h pick V).
template <typename V> struct Tiles {
    static hipError_t mfma32_factor(const LevelArgs &a, hipStream_t s)
    {
        if (a.p < 1) return hipErrorInvalidValue;
        const dim3 grid((unsigned)a.p);
        if (a.Dadd) launch_k(k_btri_mfma32<true, V>, grid, dim3(WG), s, a);
        else launch_k(k_btri_mfma32<false, V>, grid, dim3(WG), s, a);
        return hipGetLastError();
    }
    static hipError_t mfma32_factor_batch(bool add, const LevelArgs *tab, const int4 *work, int nwg,
                                          hipStream_t s)
    {
        if (nwg <= 0) return hipSuccess;
        if (add) launch_k(kb_btri_mfma32<true, V>, dim3(nwg), dim3(WG), s, tab, work);
        else launch_k(kb_btri_mfma32<false, V>, dim3(nwg), dim3(WG), s, tab, work);
        return hipGetLastError();
    }
    static hipError_t mfma16_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s)
    {
        if (a.p < 1) return hipErrorInvalidValue;
        if (sv && (sv->nrhs < 1 || sv->nrhs > 16)) return hipErrorInvalidValue;
        const dim3 grid((unsigned)a.p);
        if (sv) {
            if (a.Dadd) launch_k(k_btri_mfma16<true, true, V>, grid, dim3(WG), s, a, *sv);
            else launch_k(k_btri_mfma16<false, true, V>, grid, dim3(WG), s, a, *sv);
        } else {
            if (a.Dadd) launch_k(k_btri_mfma16<true, false, V>, grid, dim3(WG), s, a, SolveArgs{});
            else launch_k(k_btri_mfma16<false, false, V>, grid, dim3(WG), s, a, SolveArgs{});
        }
        return hipGetLastError();
    }
    static hipError_t mfma16_factor_batch(bool add, const LevelArgs *tab, const int4 *work, int nwg,
                                          hipStream_t s)
    {
        if (nwg <= 0) return hipSuccess;
        if (add) launch_k(kb_btri_mfma16<true, V>, dim3(nwg), dim3(WG), s, tab, work);
        else launch_k(kb_btri_mfma16<false, V>, dim3(nwg), dim3(WG), s, tab, work);
        return hipGetLastError();
    }
    static hipError_t babd16_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s)
    {
        if (a.p < 1) return hipErrorInvalidValue;
        if (sv && (sv->nrhs < 1 || sv->nrhs > 16)) return hipErrorInvalidValue;
        const dim3 grid((unsigned)a.p);
        if (sv) launch_k(k_babd_mfma16<true, V>, grid, dim3(WG), s, a, *sv);
        else launch_k(k_babd_mfma16<false, V>, grid, dim3(WG), s, a, SolveArgs{});
        return hipGetLastError();
    }
    static hipError_t babd16_factor_batch(const LevelArgs *tab, const int4 *work, int nwg,
                                          hipStream_t s)
    {
        if (nwg <= 0) return hipSuccess;
        launch_k(kb_babd_mfma16<V>, dim3(nwg), dim3(WG), s, tab, work);
        return hipGetLastError();
    }
    static hipError_t solvet(int M, int kind, bool fwd, bool add, const SolveArgs &a, hipStream_t s)
    {
        if (a.nrhs < 1) return hipErrorInvalidValue;
        const int cols = solve32_cols(M, sizeof(V) == 4, kind == 0 && !(fwd && add), a.nrhs, a.p);
        const dim3 grid((unsigned)a.p, (unsigned)((a.nrhs + cols - 1) / cols));
        return dispatch_T(M, [&](auto mc) {
            constexpr int MV = decltype(mc)::value;
            return dispatch_CT(cols, [&](auto ct) {
                constexpr int CT = decltype(ct)::value;
                if constexpr (MV == 32 && CT == 4 && sizeof(V) == 8) {
                    // FP64 32 x 32 blocks: 64 columns only for block
                    // tridiagonal sweeps of one right-hand side (the
                    // bidiagonal ones and an added second one would spill)
                    if (kind != 0 || (fwd && add)) return hipErrorInvalidValue;
                    if (!fwd) launch_k(k_bwdt<MV, 0, CT, V>, grid, dim3(WG), s, a);
                    else launch_k(k_fwdt<MV, 0, CT, false, V>, grid, dim3(WG), s, a);
                    return hipGetLastError();
                } else {
                    if (fwd) {
                        if (kind == 1) launch_k(k_fwdt<MV, 1, CT, false, V>, grid, dim3(WG), s, a);
                        else if (add) launch_k(k_fwdt<MV, 0, CT, true, V>, grid, dim3(WG), s, a);
                        else launch_k(k_fwdt<MV, 0, CT, false, V>, grid, dim3(WG), s, a);
                    } else {
                        if (kind == 1) launch_k(k_bwdt<MV, 1, CT, V>, grid, dim3(WG), s, a);
                        else launch_k(k_bwdt<MV, 0, CT, V>, grid, dim3(WG), s, a);
                    }
                    return hipGetLastError();
                }
            });
        });
    }
    static hipError_t solvet_batch(int M, int kind, bool fwd, bool add, int cols,
                                   const SolveArgs *tab, const int4 *work, int nwg, hipStream_t s)
    {
        if (nwg <= 0) return hipSuccess;
        return dispatch_T(M, [&](auto mc) {
            constexpr int MV = decltype(mc)::value;
            return dispatch_CT(cols, [&](auto ct) {
                constexpr int CT = decltype(ct)::value;
                if constexpr (MV == 32 && CT == 4 && sizeof(V) == 8) {
                    if (kind != 0 || (fwd && add)) return hipErrorInvalidValue;   // as in solvet
                    if (!fwd) launch_k(kb_bwdt<MV, 0, CT, V>, dim3(nwg), dim3(WG), s, tab, work);
                    else launch_k(kb_fwdt<MV, 0, CT, false, V>, dim3(nwg), dim3(WG), s, tab, work);
                    return hipGetLastError();
                } else {
                    if (fwd) {
                        if (kind == 1)
                            launch_k(kb_fwdt<MV, 1, CT, false, V>, dim3(nwg), dim3(WG), s, tab, work);
                        else if (add)
                            launch_k(kb_fwdt<MV, 0, CT, true, V>, dim3(nwg), dim3(WG), s, tab, work);
                        else
                            launch_k(kb_fwdt<MV, 0, CT, false, V>, dim3(nwg), dim3(WG), s, tab, work);
                    } else {
                        if (kind == 1) launch_k(kb_bwdt<MV, 1, CT, V>, dim3(nwg), dim3(WG), s, tab, work);
                        else launch_k(kb_bwdt<MV, 0, CT, V>, dim3(nwg), dim3(WG), s, tab, work);
                    }
                    return hipGetLastError();
                }
            });
        });
    }
};

}  // namespace
}  // namespace pf
