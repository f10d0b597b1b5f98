// Scalar tridiagonal levels (m = 1, FP64), coalesced through LDS (gfx950).
//
// A lane owns one partition (its chain of 1 x 1 blocks, Sec. 2).  Read
// straight from HBM, the 64 lanes of a wave touch 64 cache lines per
// instruction (one per partition); here the workgroup first copies its
// partitions' rows into LDS with contiguous loads, runs the chains out of
// LDS, and writes the per-row factors back with contiguous stores.  The
// stores cover every row of the workgroup's range, separators included
// (nothing reads a separator's factor row): skipping them left a partly
// written cache line every 17 rows, which cost about 40 % of the factor's
// time.  The arithmetic is that of the segment mapping with one entry per
// lane, in the same order, so both give the same bits.
#include "kernels_common.h"
#include "kernels_tri.h"

namespace pf {
namespace {

constexpr int kTriWG = 64;   // one wave; lane j owns partition 64 * blockIdx.x + j
constexpr int kStage = 9;    // staging rows in flight per lane

// A workgroup's rows: from its first partition's first block through its
// last partition's right separator (row nb for the last partition of the
// level, which the raw buffers read as zero and never write).
struct Chunk {
    int64_t c0;      // first row
    int nr;          // rows
    int64_t part0;   // first partition
};

// The balanced partition rule (partition i: q + [i < rem] blocks, then its
// right separator) from one division per workgroup.
struct Split {
    int64_t q, rem;
    __device__ __forceinline__ int64_t start(int64_t i) const { return i * (q + 1) + (i < rem ? i : rem); }
    __device__ __forceinline__ int len(int64_t i) const { return (int)(q + (i < rem ? 1 : 0)); }
};

__device__ __forceinline__ Split tri_split(int64_t nb, int64_t p)
{
    const int64_t nint = nb - (p - 1);
    Split s;
    if (nint <= 0x7FFFFFFF && p <= 0x7FFFFFFF) s.q = (int64_t)((uint32_t)nint / (uint32_t)p);
    else s.q = nint / p;
    s.rem = nint - s.q * p;
    return s;
}

__device__ __forceinline__ Chunk tri_chunk(const Split &sp, int64_t p, int64_t blk)
{
    Chunk c;
    c.part0 = blk * kTriWG;
    const int64_t last = (c.part0 + kTriWG < p ? c.part0 + kTriWG : p) - 1;
    c.c0 = sp.start(c.part0);
    c.nr = (int)(sp.start(last) + sp.len(last) + 1 - c.c0);
    return c;
}

// the lane's partition: its first row relative to the chunk, its length
// and whether it has a left / right separator
struct Lane {
    int64_t part;
    int o, len;
    bool valid, hasL, hasR;
};

__device__ __forceinline__ Lane tri_lane(const Split &sp, int64_t p, const Chunk &c, int lane)
{
    Lane l;
    l.part = c.part0 + lane;
    l.valid = l.part < p;
    l.o = l.valid ? (int)(sp.start(l.part) - c.c0) : 0;
    l.len = l.valid ? sp.len(l.part) : 0;
    l.hasL = l.valid && l.part > 0;
    l.hasR = l.valid && l.part < p - 1;
    return l;
}

// bytes of an array a staging load may read: the chunk's rows, within the
// array's n bytes from the chunk's first row
__device__ __forceinline__ uint64_t tri_span(uint64_t n, const Chunk &c)
{
    const uint64_t w = (uint64_t)c.nr * 8;
    return n < w ? n : w;
}

__device__ __forceinline__ double prod(double u, double v)
{
    const double a[1] = {u}, b[1] = {v};
    return dot<1, double>(a, b);
}

// Factor (and with RHS the forward sweep) of one level.  KM: the longest
// chain the LDS arrays hold.
template <int KM, bool ADD, bool RHS>
__global__ __launch_bounds__(kTriWG) void k_tri_factor(LevelArgs a, SolveArgs sv)
{
    constexpr int NR = kTriWG * (KM + 1);
    __shared__ double sD[NR], sL[NR], sU[NR], sR[NR];
    __shared__ double sF[RHS ? NR : 1];
    const int lane = threadIdx.x;
    const int64_t nb = a.nb, p = a.p;
    const Split sp = tri_split(nb, p);
    const Chunk c = tri_chunk(sp, p, blockIdx.x);

    // raw buffers based at the chunk's first row: rows past an array's end
    // take no stores, and loads past the chunk or the array read zero
    // without touching memory
    const uint64_t n0 = (uint64_t)(nb - c.c0) * 8;
    const uint64_t n1 = nb - 1 > c.c0 ? (uint64_t)(nb - 1 - c.c0) * 8 : 0;
    const uint64_t m0 = tri_span(n0, c), m1 = tri_span(n1, c);
    const auto rD = buf_rsrc(a.D + c.c0, m0);
    const auto rDa = buf_rsrc(ADD ? a.Dadd + c.c0 : a.D, ADD ? m0 : 0);
    const auto rL = buf_rsrc(a.Lo + c.c0, m1);
    const auto rU = buf_rsrc(a.Up + c.c0, m1);
    const auto rF = buf_rsrc(RHS ? sv.F + c.c0 : a.D, RHS ? m0 : 0);
    const auto rFa = buf_rsrc((RHS && ADD) ? sv.Fadd + c.c0 : a.D, (RHS && ADD) ? m0 : 0);

    // stage D (+ Dadd), A(g+1,g), A(g,g+1) and f (+ Fadd): kStage rows in
    // flight per lane, each instruction reading 64 consecutive rows
    for (int i0 = 0; i0 < c.nr; i0 += kStage * kTriWG) {
        double d[kStage], l[kStage], u[kStage], f[kStage];
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const uint32_t o = (uint32_t)(i0 + k * kTriWG + lane) * 8u;
            d[k] = buf_ld(rD, o);
            if constexpr (ADD) d[k] += buf_ld(rDa, o);
            l[k] = buf_ld(rL, o);
            u[k] = buf_ld(rU, o);
            f[k] = 0.0;
            if constexpr (RHS) {
                f[k] = buf_ld(rF, o);
                if constexpr (ADD) f[k] += buf_ld(rFa, o);
            }
        }
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const int i = i0 + k * kTriWG + lane;
            if (i < c.nr) {
                sD[i] = d[k];
                sL[i] = l[k];
                sU[i] = u[k];
                if constexpr (RHS) sF[i] = f[k];
            }
        }
    }
    wave_sync();

    // the chain of partition `part`; the rows it reads and writes are its
    // own, apart from its right separator's D and f (read only) and its left
    // separator's couplings (read only, at local row o - 1)
    const Lane G = tri_lane(sp, p, c, lane);
    const int64_t part = G.part, g0 = c.c0 + G.o;
    const int o = G.o;
    double d = 0.0, fp = 0.0, z = 0.0, rr = 0.0, a1 = 0.0, gl = 0.0;
    if (G.valid) {
        d = sD[o];
        if constexpr (RHS) fp = sF[o];
    }
    if (G.hasL) {
        if (lane == 0) {   // the previous workgroup's separator
            z = a.Lo[g0 - 1];
            rr = a.Up[g0 - 1];
        } else {
            z = sL[o - 1];
            rr = sU[o - 1];
        }
    }
    unsigned long long bad = ~0ull;
    double up = sU[o], lo = sL[o], dn = sD[o + 1], fn = RHS ? sF[o + 1] : 0.0;
    for (int k = 0; k < G.len; ++k) {
        const int i = o + k;
        const double cu = up, cl = lo, cd = dn, cf = fn;
        if (k + 1 < G.len) {
            up = sU[i + 1];
            lo = sL[i + 1];
            dn = sD[i + 2];
            if constexpr (RHS) fn = sF[i + 2];
        }
        const unsigned long long code = status_code(a.level, g0 + k);
        bad = (d == 0.0 && code < bad) ? code : bad;
        const double e = recip(d);             // E_k = D'_k^{-1}
        const double x = prod(e, cu);          // X_k = E_k A(g,g+1)
        const double zh = prod(e, z);          // Zh_k = E_k Z'_k
        const double tk = RHS ? prod(e, fp) : 0.0;   // t_k = E_k f'_k
        sD[i] = e;
        sU[i] = x;
        sL[i] = zh;
        sR[i] = rr;
        if constexpr (RHS) sF[i] = tk;
        a1 -= prod(rr, zh);                    // alpha_1 -= R_k Zh_k
        const double rn = -prod(rr, x);        // R_{k+1} = -R_k X_k
        d = cd - prod(cl, x);                  // D'_{k+1} = D_{g+1} - A(g+1,g) X_k
        z = -prod(cl, zh);                     // Z'_{k+1} = -A(g+1,g) Zh_k
        if constexpr (RHS) {
            gl -= prod(rr, tk);                // g_sL -= R_k t_k
            fp = cf - prod(cl, tk);            // f'_{k+1} = f_{g+1} - A(g+1,g) t_k
        }
        rr = rn;
    }
    if (G.valid) sR[o + G.len] = 0.0;   // the right separator's row (no factor)
    report_bad(a, bad);
    if (G.hasR) {
        a.nD[part] = d;                        // D[sR] + alpha_2
        if (G.hasL) a.nLo[part - 1] = z;       // beta
    }
    if (G.hasL) {
        a.nDadd[part - 1] = a1;                // alpha_1
        if (G.hasR) a.nUp[part - 1] = rr;      // gamma
    }
    if constexpr (RHS) {
        if (G.hasR) sv.nF[part] = fp;          // f[sR] - A(sR,g_n) t_n
        if (G.hasL) sv.nFadd[part - 1] = gl;   // - sum R_k t_k
    }
    wave_sync();

    // factors, contiguous.  The separators' rows are written too (with what
    // LDS holds there; nothing reads them) so that stores cover whole cache
    // lines; partition 0's R rows hold zero.
    const auto rE = buf_rsrc((double *)a.E + c.c0, n0);
    const auto rX = buf_rsrc((double *)a.X + c.c0, n0);
    const auto rZ = buf_rsrc((double *)a.Z + c.c0, n0);
    const auto rR = buf_rsrc((double *)a.R + c.c0, n0);
    const auto rY = buf_rsrc(RHS ? sv.Y + c.c0 : (double *)a.dump, RHS ? n0 : 0);
    for (int i = lane; i < c.nr; i += kTriWG) {
        const uint32_t off = (uint32_t)i * 8u;
        buf_st(rE, off, sD[i]);
        buf_st(rX, off, sU[i]);
        buf_st(rZ, off, sL[i]);
        buf_st(rR, off, sR[i]);
        if constexpr (RHS) buf_st(rY, off, sF[i]);
    }
}

// Forward sweep of one level (one right-hand side) with stored factors:
// t_k = E_k f'_k, f'_{k+1} = f_{g+1} - A(g+1,g) t_k, g_sL -= R_k t_k.
template <int KM, bool ADD>
__global__ __launch_bounds__(kTriWG) void k_tri_fwd(SolveArgs a)
{
    constexpr int NR = kTriWG * (KM + 1);
    __shared__ double sE[NR], sR[NR], sL[NR], sF[NR];
    const int lane = threadIdx.x;
    const int64_t nb = a.nb, p = a.p;
    const Split sp = tri_split(nb, p);
    const Chunk c = tri_chunk(sp, p, blockIdx.x);
    const uint64_t n0 = (uint64_t)(nb - c.c0) * 8;
    const uint64_t n1 = nb - 1 > c.c0 ? (uint64_t)(nb - 1 - c.c0) * 8 : 0;
    const uint64_t m0 = tri_span(n0, c), m1 = tri_span(n1, c);
    const auto rE = buf_rsrc((const double *)a.E + c.c0, m0);
    const auto rR = buf_rsrc((const double *)a.R + c.c0, m0);
    const auto rL = buf_rsrc(a.Lo + c.c0, m1);
    const auto rF = buf_rsrc(a.F + c.c0, m0);
    const auto rFa = buf_rsrc(ADD ? a.Fadd + c.c0 : a.F, ADD ? m0 : 0);
    for (int i0 = 0; i0 < c.nr; i0 += kStage * kTriWG) {
        double e[kStage], r[kStage], l[kStage], f[kStage];
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const uint32_t o = (uint32_t)(i0 + k * kTriWG + lane) * 8u;
            e[k] = buf_ld(rE, o);
            r[k] = buf_ld(rR, o);
            l[k] = buf_ld(rL, o);
            f[k] = buf_ld(rF, o);
            if constexpr (ADD) f[k] += buf_ld(rFa, o);
        }
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const int i = i0 + k * kTriWG + lane;
            if (i < c.nr) {
                sE[i] = e[k];
                sR[i] = r[k];
                sL[i] = l[k];
                sF[i] = f[k];
            }
        }
    }
    wave_sync();
    const Lane G = tri_lane(sp, p, c, lane);
    const int o = G.o;
    double fp = G.valid ? sF[o] : 0.0, gl = 0.0;
    for (int k = 0; k < G.len; ++k) {
        const int i = o + k;
        const double t = prod(sE[i], fp);      // t_k
        const double rr = G.hasL ? sR[i] : 0.0;   // partition 0 stores no R
        const double fn = sF[i + 1];
        sF[i] = t;
        fp = fn - prod(sL[i], t);
        gl -= prod(rr, t);
    }
    if (G.hasR) a.nF[G.part] = fp;
    if (G.hasL) a.nFadd[G.part - 1] = gl;
    wave_sync();
    const auto rY = buf_rsrc(a.Y + c.c0, n0);
    for (int i = lane; i < c.nr; i += kTriWG)
        buf_st(rY, (uint32_t)i * 8u, sF[i]);   // separators: their f, overwritten by x later
}

// Back substitution of one level (one right-hand side):
// x_k = t_k - Zh_k x_sL - X_k x_{k+1}, from the partition's last row up.
template <int KM>
__global__ __launch_bounds__(kTriWG) void k_tri_bwd(SolveArgs a)
{
    constexpr int NR = kTriWG * (KM + 1);
    __shared__ double sZ[NR], sX[NR], sT[NR];
    const int lane = threadIdx.x;
    const int64_t nb = a.nb, p = a.p;
    const Split sp = tri_split(nb, p);
    const Chunk c = tri_chunk(sp, p, blockIdx.x);
    const uint64_t n0 = (uint64_t)(nb - c.c0) * 8, m0 = tri_span(n0, c);
    const auto rZ = buf_rsrc((const double *)a.Z + c.c0, m0);
    const auto rX = buf_rsrc((const double *)a.X + c.c0, m0);
    const auto rT = buf_rsrc(a.Y + c.c0, m0);
    const auto rY = buf_rsrc(a.Y + c.c0, n0);
    for (int i0 = 0; i0 < c.nr; i0 += kStage * kTriWG) {
        double z[kStage], x[kStage], t[kStage];
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const uint32_t o = (uint32_t)(i0 + k * kTriWG + lane) * 8u;
            z[k] = buf_ld(rZ, o);
            x[k] = buf_ld(rX, o);
            t[k] = buf_ld(rT, o);
        }
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const int i = i0 + k * kTriWG + lane;
            if (i < c.nr) {
                sZ[i] = z[k];
                sX[i] = x[k];
                sT[i] = t[k];
            }
        }
    }
    const Lane G = tri_lane(sp, p, c, lane);
    const int64_t part = G.part;
    const int o = G.o;
    const double xl = G.hasL ? a.Xsep[part - 1] : 0.0;
    const double xr = G.hasR ? a.Xsep[part] : 0.0;
    wave_sync();
    if (G.hasR) sT[o + G.len] = xr;            // the right separator's solution
    double xn = xr;
    for (int k = G.len - 1; k >= 0; --k) {
        const int i = o + k;
        const double s = fma(-sX[i], xn, fma(-sZ[i], xl, sT[i]));
        sT[i] = s;
        xn = s;
    }
    wave_sync();
    for (int i = lane; i < c.nr; i += kTriWG) buf_st(rY, (uint32_t)i * 8u, sT[i]);
}

int tri_kmax(int64_t nb, int64_t p)
{
    const int64_t nint = nb - (p - 1);
    return (int)(nint / p + (nint % p ? 1 : 0));
}

// LDS arrays sized for the level's longest chain (5, 9, 13 or 17 blocks):
// the smaller they are, the more workgroups share a compute unit
template <typename F>
void dispatch_km(int64_t nb, int64_t p, F &&f)
{
    const int k = tri_kmax(nb, p);
    if (k <= 5) f(std::integral_constant<int, 5>{});
    else if (k <= 9) f(std::integral_constant<int, 9>{});
    else if (k <= 13) f(std::integral_constant<int, 13>{});
    else f(std::integral_constant<int, kTriMaxChain>{});
}

}  // namespace

bool tri_fits(int64_t nb, int64_t p)
{
    return p >= 1 && nb >= 2 && p <= (nb + 1) / 2 && tri_kmax(nb, p) <= kTriMaxChain;
}

hipError_t launch_tri_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s)
{
    if (!tri_fits(a.nb, a.p)) return hipErrorInvalidValue;
    if (sv && sv->nrhs != 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.p + kTriWG - 1) / kTriWG));
    const SolveArgs none{};
    const SolveArgs &v = sv ? *sv : none;
    const bool add = a.Dadd != nullptr;
    dispatch_km(a.nb, a.p, [&](auto km) {
        constexpr int K = decltype(km)::value;
        if (add) {
            if (sv) launch_k((k_tri_factor<K, true, true>), grid, dim3(kTriWG), s, a, v);
            else launch_k((k_tri_factor<K, true, false>), grid, dim3(kTriWG), s, a, v);
        } else {
            if (sv) launch_k((k_tri_factor<K, false, true>), grid, dim3(kTriWG), s, a, v);
            else launch_k((k_tri_factor<K, false, false>), grid, dim3(kTriWG), s, a, v);
        }
    });
    return hipGetLastError();
}

hipError_t launch_tri_fwd(const SolveArgs &a, hipStream_t s)
{
    if (!tri_fits(a.nb, a.p) || a.nrhs != 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.p + kTriWG - 1) / kTriWG));
    dispatch_km(a.nb, a.p, [&](auto km) {
        constexpr int K = decltype(km)::value;
        if (a.Fadd) launch_k((k_tri_fwd<K, true>), grid, dim3(kTriWG), s, a);
        else launch_k((k_tri_fwd<K, false>), grid, dim3(kTriWG), s, a);
    });
    return hipGetLastError();
}

hipError_t launch_tri_bwd(const SolveArgs &a, hipStream_t s)
{
    if (!tri_fits(a.nb, a.p) || a.nrhs != 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.p + kTriWG - 1) / kTriWG));
    dispatch_km(a.nb, a.p, [&](auto km) {
        launch_k((k_tri_bwd<decltype(km)::value>), grid, dim3(kTriWG), s, a);
    });
    return hipGetLastError();
}

}  // namespace pf
