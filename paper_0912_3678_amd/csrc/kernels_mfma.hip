// Partition-method factor kernel for 8 x 8 blocks with the block products on
// the matrix cores (gfx950, FP64, block tridiagonal, finest level).
//
// Two partitions share a wave.  Their pivot blocks are inverted by the
// Gauss-Jordan exchange steps of kernels_gj.h with two entries per lane (the
// "inversion role" of a lane: partition tid / 32, entries (r, 2g), (r, 2g+1)).
// The block products of a chain row -- X = E A(g,g+1), Zh = E Z', t = E f',
// D'_{k+1}, Z'_{k+1}, f'_{k+1} and the spike-row updates -- run as pairs of
// v_mfma_f64_16x16x4f64 with the two partitions' 8 x 8 blocks on the diagonal
// of the 16 x 16 tile, so their operands stay in registers (the products of
// the segment mapping stream rows and columns through LDS, which bounds that
// kernel).
//
// Matrix-core role of lane l: partition p = bit 3 of l; of an 8 x 8 matrix Y
// of its partition the lane holds the "pair" Y(m, c), Y(m + 4, c) with
// m = l >> 4, c = l & 7.  For C = A B of both partitions, instruction h
// (h = 0, 1) takes at lane l the A operand A(c, 4h + m) and the B operand
// B(4h + m, c) -- entry h of the pair of A^T and of B -- and leaves
// C(m + 4q, c) in result register 2p + q.  A result therefore feeds the next
// product as its right operand, and as the left operand of a transposed
// product: the spike rows are carried transposed (R^T, alpha_1^T, g^T).  The
// inverse enters through LDS (its transpose's pair read from the logical rows
// the exchange steps leave) and D' goes back to the inversion layout through
// LDS.  The recurrences and outputs are those of the other factor kernels.
#include "kernels_gj.h"

namespace pf {
namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

// C + A B for both partitions; a = pair of A^T, b = pair of B
__device__ __forceinline__ dv4 mm2(const double (&a)[2], const double (&b)[2], dv4 c)
{
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
}
// the lane's partition's pair out of a result
__device__ __forceinline__ void pair_of(const dv4 &d, bool p1, double (&y)[2])
{
    y[0] = p1 ? d[2] : d[0];
    y[1] = p1 ? d[3] : d[1];
}
// a pair as the accumulator input (both partitions' result registers)
__device__ __forceinline__ dv4 acc_of(const double (&y)[2])
{
    dv4 c;
    c[0] = y[0]; c[1] = y[1]; c[2] = y[0]; c[3] = y[1];
    return c;
}
__device__ __forceinline__ void neg2(const double (&y)[2], double (&z)[2])
{
    z[0] = -y[0];
    z[1] = -y[1];
}

template <bool RHS>
__device__ __forceinline__ void btri_mfma_body(const LevelArgs &a, const SolveArgs &sv,
                                               int64_t pblock)
{
    constexpr int M = 8, E = 2, LP = 32, PPW = 2, PD = 1;
    constexpr size_t MM = 64;
    constexpr int RS = M + kPad<double>;
    constexpr uint32_t BB = MM * 8;
    const int tid = threadIdx.x;
    // inversion role
    const int gp = tid / LP, t = tid % LP, r = t % M, gc = t / M, c0 = gc * E;
    // matrix-core role
    const int mp = (tid >> 3) & 1, m = tid >> 4, c = tid & 7;
    const bool p1 = mp == 1;

    constexpr int SL = M * RS;
    constexpr int GS = group_stride<double>(3 * SL);
    __shared__ __align__(16) double lds[PPW * GS];
    double *S0g = lds + gp * GS;        // inversion role: tableau
    double *SEg = S0g + SL;             //   E by logical rows
    double *SDg = SEg + SL;             //   D' handed over
    double *SEm = lds + mp * GS + SL;   // matrix-core role: E
    double *SDm = SEm + SL;             //   D'

    // The wave's partitions.  A partition past the last one shadows the first
    // (same rows, every output dropped), so both have lengths within one.
    const int64_t nb = a.nb;
    const Geo G0 = geometry_wave<0>(nb, a.p, pblock * PPW, a.sep);
    const Geo G1r = geometry_wave<0>(nb, a.p, pblock * PPW + 1, a.sep);
    const bool sh1 = !G1r.valid;
    const Geo G1 = sh1 ? G0 : G1r;
    const Geo &Gg = gp ? G1 : G0, &Gm = mp ? G1 : G0;
    const bool outg = !(gp && sh1), outm = !(mp && sh1);   // role's outputs are kept
    const int64_t part_m = pblock * PPW + mp;
    const int kmin = G0.len < G1.len ? G0.len : G1.len;
    const int kmax = G0.len < G1.len ? G1.len : G0.len;

    const int64_t gb = G0.start > 0 ? G0.start - 1 : 0;
    const uint64_t nr = (uint64_t)(nb - gb), nr1 = nb - 1 > gb ? (uint64_t)(nb - 1 - gb) : 0;
    const auto rD = buf_rsrc(a.D + gb * MM, nr * BB);
    const auto rL = buf_rsrc(a.Lo + gb * MM, nr1 * BB);
    const auto rU = buf_rsrc(a.Up + gb * MM, nr1 * BB);
    const auto rE = buf_rsrc((double *)a.E + gb * MM, nr * BB);
    const auto rR = buf_rsrc((double *)a.R + gb * MM, nr * BB);
    const auto rZ = buf_rsrc((double *)a.Z + gb * MM, nr * BB);
    const auto rX = buf_rsrc((double *)a.X + gb * MM, nr * BB);
    const uint32_t relg = (uint32_t)(Gg.start - gb), relm = (uint32_t)(Gm.start - gb);
    // byte offsets inside a column-major block: the pair (m + 4h, c) at
    // opair + 32h, the pair of the transpose (c, m + 4h) at otr + 256h
    const uint32_t opair = (uint32_t)(m + 8 * c) * 8, otr = (uint32_t)(c + 8 * m) * 8;
    // inside a row-major factor block: pair (m + 4h, c) at fpair + 256h,
    // transposed pair (c, m + 4h) at ftr + 32h
    const uint32_t fpair = (uint32_t)(8 * m + c) * 8, ftr = (uint32_t)(8 * c + m) * 8;

    double *ydump = (double *)a.dump + 2048 + tid * 2;
    const double *zero = a.zero;
    const bool act = RHS && c < sv.nrhs;   // right-hand-side column c of the pairs
    const int64_t fo = (int64_t)m + (int64_t)(act ? c : 0) * sv.ldf;
    const int64_t yo = (int64_t)m + (int64_t)(act ? c : 0) * sv.ldy;

    // state: D' (inversion layout); Z', R^T, alpha_1^T, f', g^T (pairs)
    double d[2], dp[2], z[2], rT[2], a1[2], f[2], gt[2];
    {
        const uint32_t o = relg * BB + (uint32_t)(r + 8 * c0) * 8;
        d[0] = buf_ld(rD, o);
        d[1] = buf_ld(rD, o + 64);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        dp[h] = 0.0;
        a1[h] = 0.0;
        gt[h] = 0.0;
        z[h] = Gm.hasL ? buf_ld(rL, (relm - 1) * BB + opair + 32 * h) : 0.0;   // Z'_1 = A(g_1, sL)
        rT[h] = Gm.hasL ? buf_ld(rU, (relm - 1) * BB + otr + 256 * h) : 0.0;   // R_1 = A(sL, g_1)
        f[h] = (RHS && act && Gm.valid) ? sv.F[Gm.start * M + fo + 4 * h] : 0.0;
    }
    unsigned long long bad = ~0ull;

    // operands of block row g (matrix-core role), PD rows ahead (one row: the
    // inversion covers the latency, and fewer registers stay live): pairs of
    // A(g,g+1), of A(g+1,g)^T, of D[g+1] and of f[g+1]
    struct Next {
        double up[2], lo[2], dn[2], fn[2];
    };
    auto load_next = [&](int k, Next &n) {
        const uint32_t row = relm + (uint32_t)k;
        const int64_t g = Gm.start + k;
        const bool okf = act && k < Gm.len && g + 1 < nb;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            n.up[h] = buf_ld(rU, row * BB + opair + 32 * h);
            n.lo[h] = buf_ld(rL, row * BB + otr + 256 * h);
            n.dn[h] = buf_ld(rD, (row + 1) * BB + opair + 32 * h);
            n.fn[h] = RHS ? *(okf ? sv.F + (g + 1) * M + fo + 4 * h : zero) : 0.0;
        }
    };
    Next buf[PD + 1];
#pragma unroll
    for (int q = 0; q < PD; ++q) load_next(q, buf[q]);

    // one block row; MASK: a partition may have ended (its state is kept and
    // its stores dropped)
    auto row = [&](auto maskc, int k) {
        constexpr bool MASK = decltype(maskc)::value;
        const bool lg = !MASK || k < Gg.len, lm = !MASK || k < Gm.len;
        const bool sg = lg && outg, sm = lm && outm;   // stores kept
        load_next(k + PD, buf[PD]);
        const Next &cur = buf[0];

        // E_k = D'_k^{-1} (inversion role)
        double b[2] = {d[0], d[1]};
        int sigma = 0, pc[2] = {0, 0};
        bool sing = false;
        seg_invert<M, E, double>(b, r, gc, S0g, sigma, pc, sing);
        const unsigned long long code = status_code(a.level, Gg.start + k);
        bad = (sing && sg && code < bad) ? code : bad;
        const uint32_t frg = (relg + (uint32_t)k) * BB;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            SEg[sigma * RS + pc[e]] = b[e];
            buf_st(rE, sg ? frg + (uint32_t)(sigma * M + pc[e]) * 8 : kOffNone, b[e]);
        }
        wave_sync();

        // products (matrix-core role)
        const double eT[2] = {SEm[c * RS + m], SEm[c * RS + m + 4]};
        const dv4 zero4 = {0.0, 0.0, 0.0, 0.0};
        double x[2], zh[2], tt[2] = {0.0, 0.0};
        pair_of(mm2(eT, cur.up, zero4), p1, x);    // X_k = E_k A(g,g+1)
        pair_of(mm2(eT, z, zero4), p1, zh);        // Zh_k = E_k Z'_k
        if constexpr (RHS) pair_of(mm2(eT, f, zero4), p1, tt);   // t_k = E_k f'_k
        double nlo[2], nx[2], nzh[2];
        neg2(cur.lo, nlo);
        neg2(x, nx);
        neg2(zh, nzh);
        double dn[2], zn[2], rn[2], an[2], fnw[2], gn[2];
        pair_of(mm2(nlo, x, acc_of(cur.dn)), p1, dn);   // D'_{k+1} = D[g+1] - A(g+1,g) X_k
        pair_of(mm2(nlo, zh, zero4), p1, zn);           // Z'_{k+1} = -A(g+1,g) Zh_k
        pair_of(mm2(nx, rT, zero4), p1, rn);            // R_{k+1}^T = -X_k^T R_k^T
        pair_of(mm2(nzh, rT, acc_of(a1)), p1, an);      // alpha_1^T -= Zh_k^T R_k^T
        if constexpr (RHS) {
            double nt[2];
            neg2(tt, nt);
            pair_of(mm2(nlo, tt, acc_of(cur.fn)), p1, fnw);   // f'_{k+1} = f[g+1] - A(g+1,g) t_k
            pair_of(mm2(nt, rT, acc_of(gt)), p1, gn);         // g^T -= t_k^T R_k^T
        }

        // factors of row k: X, Zh, R_k (row-major), t
        const uint32_t frm = (relm + (uint32_t)k) * BB;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            buf_st(rX, sm ? frm + fpair + 256 * h : kOffNone, x[h]);
            buf_st(rZ, sm ? frm + fpair + 256 * h : kOffNone, zh[h]);
            buf_st(rR, (sm && Gm.hasL) ? frm + ftr + 32 * h : kOffNone, rT[h]);
            if constexpr (RHS)
                *((sm && act) ? sv.Y + (Gm.start + k) * M + yo + 4 * h : ydump + h) = tt[h];
        }

        // state
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            dp[h] = (MASK && !lm) ? dp[h] : dn[h];
            z[h] = (MASK && !lm) ? z[h] : zn[h];
            rT[h] = (MASK && !lm) ? rT[h] : rn[h];
            a1[h] = (MASK && !lm) ? a1[h] : an[h];
            if constexpr (RHS) {
                f[h] = (MASK && !lm) ? f[h] : fnw[h];
                gt[h] = (MASK && !lm) ? gt[h] : gn[h];
            }
        }
        // D'_{k+1} to the inversion layout
        SDm[m * RS + c] = dn[0];
        SDm[(m + 4) * RS + c] = dn[1];
        wave_sync();
        double dd[2];
        lds_get<2, double>(dd, SDg + r * RS + c0);
        d[0] = (MASK && !lg) ? d[0] : dd[0];
        d[1] = (MASK && !lg) ? d[1] : dd[1];
#pragma unroll
        for (int q = 0; q < PD; ++q) buf[q] = buf[q + 1];
        wave_sync();
    };
    int k = 0;
    for (; k < kmin; ++k) row(std::integral_constant<bool, false>{}, k);
    if (k < kmax) row(std::integral_constant<bool, true>{}, k);

    report_bad(a, bad);
    if (Gm.valid && outm) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cm = m + 4 * h + c * M;    // (m + 4h, c), column-major
            const int ct = c + (m + 4 * h) * M;  // (c, m + 4h), column-major
            if (Gm.hasR) {
                a.nD[part_m * MM + cm] = dp[h];                       // D[sR] + alpha_2
                if (Gm.hasL) a.nLo[(part_m - 1) * MM + cm] = z[h];    // beta
            }
            if (Gm.hasL) {
                a.nDadd[(part_m - 1) * MM + ct] = a1[h];              // alpha_1
                if (Gm.hasR) a.nUp[(part_m - 1) * MM + ct] = rT[h];   // gamma
            }
            if constexpr (RHS) {
                if (Gm.hasR && act)
                    sv.nF[part_m * M + m + 4 * h + (int64_t)c * sv.ldn] = f[h];   // f[sR] - A(sR,g_n) t_n
                if (Gm.hasL && m + 4 * h < sv.nrhs)
                    sv.nFadd[(part_m - 1) * M + c + (int64_t)(m + 4 * h) * sv.ldn] = gt[h];   // -sum R_k t_k
            }
        }
    }
}

template <bool RHS>
__global__ __launch_bounds__(WG) void k_btri_mfma(LevelArgs a, SolveArgs sv)
{
    btri_mfma_body<RHS>(a, sv, blockIdx.x);
}
// batched (factor only): workgroup w serves table entry work[w].x, partition
// block work[w].y
__global__ __launch_bounds__(WG) void kb_btri_mfma(const LevelArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    btri_mfma_body<false>(a, SolveArgs{}, w.y);
}

}  // namespace

bool mfma_ok(int kind, int M, bool f32, bool add)
{
    return kind == 0 && M == 8 && !f32 && !add;
}

int mfma_partitions_per_wg() { return 2; }

hipError_t launch_mfma_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s)
{
    if (sv && (sv->nrhs < 1 || sv->nrhs > 8)) return hipErrorInvalidValue;
    if (a.p < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.p + 1) / 2));
    if (sv) launch_k(k_btri_mfma<true>, grid, dim3(WG), s, a, *sv);
    else launch_k(k_btri_mfma<false>, grid, dim3(WG), s, a, SolveArgs{});
    return hipGetLastError();
}

hipError_t launch_mfma_factor_batch(const LevelArgs *tab, const int4 *work, int nwg, hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    launch_k(kb_btri_mfma, dim3(nwg), dim3(WG), s, tab, work);
    return hipGetLastError();
}

}  // namespace pf
