// Helpers shared by the partition-method kernels (gfx950, wave64).
//
// A workgroup is one wave64 and a partition never leaves its wave, so the
// only ordering needed between an LDS write and the reads of other lanes is
// the in-order LDS pipe of the wave plus a compiler fence (wave_sync); no
// workgroup barrier is used.
//
// Memory discipline inside the chain loops: no memory operation sits under
// a branch (missing operands are read from a zero block, stores a lane must
// not make go to a dump buffer, the zero-pivot report is deferred), and the
// operands of the next block row are loaded before the current row's
// stores.  The compiler's wait counters then stay exact and a row never waits
// for the stores of the previous one (loads and stores share one in-order
// counter on this architecture).
#pragma once
#include "pf_internal.h"

#include <hip/hip_ext.h>

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
// the first (count mod p) partitions getting one block more.  With an
// explicit separator list sep (p + 1 entries: partition i covers the blocks
// sep[i] + 1 .. sep[i + 1] - 1; for block tridiagonal levels sep[0] = -1 and
// sep[p] = nb stand for the ends, for the bidiagonal-plus-corner form both
// ends are real separators) the partitions are the ranges between them --
// a level whose reduced system was enlarged by blocks the elimination could
// not pivot on; a partition may then be empty.
struct Geo {
    int64_t start;   // first block of the partition
    int len;         // blocks in the partition
    int kmax;        // longest partition (uniform loop bound)
    bool valid, hasL, hasR;
};

template <int KIND>
__device__ __forceinline__ Geo geometry(int64_t nb, int64_t p, int64_t part,
                                        const int64_t *sep = nullptr)
{
    Geo g;
    g.valid = part < p;
    if (sep) {
        const int64_t pp = g.valid ? part : p - 1;
        g.start = sep[pp] + 1;
        g.len = g.valid ? (int)(sep[pp + 1] - sep[pp] - 1) : 0;
        g.kmax = g.len;
    } else {
        const int64_t nint = (KIND == 0) ? nb - (p - 1) : nb - (p + 1);
        const int64_t q = nint / p, rem = nint % p;
        const int64_t mn = part < rem ? part : rem;
        g.start = (KIND == 0 ? 0 : 1) + part * (q + 1) + mn;
        g.len = g.valid ? (int)(q + (part < rem ? 1 : 0)) : 0;
        g.kmax = (int)(q + (rem > 0 ? 1 : 0));
    }
    if (KIND == 0) {
        g.hasL = g.valid && part > 0;
        g.hasR = g.valid && part < p - 1;
    } else {
        g.hasL = g.valid;
        g.hasR = g.valid;
    }
    return g;
}

// The geometry of a partition that is the same in every lane of the wave
// (one partition per wave, or the first of a workgroup's): taken from the
// first lane, so that what is built from it -- buffer descriptors above all
// -- stays in scalar registers.  (Read from an explicit separator list, the
// values come from a vector load, which the compiler cannot know to be
// uniform; a descriptor built from them would otherwise be rebuilt lane by
// lane around every buffer access.)
template <int KIND>
__device__ __forceinline__ Geo geometry_wave(int64_t nb, int64_t p, int64_t part,
                                             const int64_t *sep)
{
    Geo g = geometry<KIND>(nb, p, part, sep);
    // on every path: a value merged from the list's branch counts as
    // non-uniform whichever branch ran
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)g.start);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)g.start >> 32));
    g.start = (int64_t)(((uint64_t)hi << 32) | lo);
    g.len = __builtin_amdgcn_readfirstlane(g.len);
    g.kmax = __builtin_amdgcn_readfirstlane(g.kmax);
    return g;
}

// A partition's pivot-block failures: the first one (smallest level and
// block) goes to the status word; with a list (enlarged reduced systems)
// every failing partition also appends its first failing block, which the
// host turns into a separator.  Called by every lane of the partition with
// the same code (the host removes the repeats).
template <class LA>
__device__ __forceinline__ void report_bad(const LA &a, unsigned long long bad)
{
    if (bad == ~0ull) return;
    atomicMin(a.status, bad);
    if (a.badlist) {
        const unsigned i = atomicAdd(a.badcount, 1u);
        if (i < (unsigned)a.badcap) a.badlist[i] = bad;
    }
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

// ---- raw buffers -----------------------------------------------------------
// A raw buffer resource over [base, base + bytes): loads at byte offsets at or
// past the end return zero and stores there are dropped (the hardware range
// check of raw buffers, which covers the per-lane offset).  Offsets are 32
// bits, so kernels rebase a resource per workgroup near the rows it touches.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint64_t bytes)
{
    const uint32_t n = bytes > 0xFFFFFF00ull ? 0xFFFFFF00u : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n, 0x00020000);
}
// an offset past the end of every resource (sizes are clamped below it): a
// store there is dropped
constexpr uint32_t kOffNone = 0xFFFFFFF0u;

__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                          r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}
// E consecutive T at byte offset off (16-byte stores where the size allows)
template <int E, typename T>
__device__ __forceinline__ void buf_st_row(__amdgpu_buffer_rsrc_t r, uint32_t off, const T (&v)[E])
{
    if constexpr (sizeof(T) == 8 && E % 2 == 0) {
        using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
#pragma unroll
        for (int e = 0; e < E; e += 2) {
            const double2 w = make_double2(v[e], v[e + 1]);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, w), r, (int)(off + e * 8), 0, 0);
        }
    } else if constexpr (sizeof(T) == 4 && E % 4 == 0) {
        using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
#pragma unroll
        for (int e = 0; e < E; e += 4) {
            const float4 w = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, w), r, (int)(off + e * 4), 0, 0);
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) buf_st(r, off + e * (uint32_t)sizeof(T), v[e]);
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
    return KC == 1 ? f(std::integral_constant<int, 1>{})
           : KC == 4 ? f(std::integral_constant<int, 4>{}) : f(std::integral_constant<int, 8>{});
}

inline dim3 grid_for(int M, int64_t p, int nrhs, int KC)
{
    const int64_t gpw = WG / M;
    return dim3((unsigned)((p + gpw - 1) / gpw), (unsigned)((nrhs + KC - 1) / KC), 1);
}

// Launch a kernel on stream s; when launch_timing() holds events, the
// kernel's own start and end are stamped into them (and they are consumed).
template <typename K, typename... Args>
inline void launch_k(K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args)
{
    LaunchTiming &t = launch_timing();
    if (t.start) {
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t.start, t.stop, 0, args...);
        t.start = t.stop = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    }
}

}  // namespace
}  // namespace pf
